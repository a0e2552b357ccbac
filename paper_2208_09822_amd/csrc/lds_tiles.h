// Block kernels of the generated family that read their operands from LDS.
//
// The batched kernel stages each problem's A and B into LDS as verbatim
// copies of their memory spans (same leading dimensions, no reordering: the
// copy is a contiguous stream of 16-byte loads, not a pack), then every
// wavefront of the work-group computes one block of the problem's tile plan
// from LDS.  Each scheme performs exactly the floating-point operations of
// its direct-from-memory counterpart in tiles.h, in the same order, so a
// problem gives bitwise the same C through either path.
//
// C is staged with A and B (when beta != 0), so a block never waits on
// memory: it reads everything from LDS and only stores.  `sync` says how a
// block waits for the staging copies before reading LDS (the batched kernel
// waits once per batch, so it passes SYNC_NONE).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tiles.h"

namespace iaat {
namespace dev {

typedef __attribute__((address_space(3))) float lds_f;

// A staged problem: la/lb/lc point at the first element of the staged A /
// B / C; element (r, c) of a stored matrix sits at la[r + c*lda] (resp. lb,
// lc with ldb, ldc).  lc is null when C is not read (beta == 0).
struct LdsProb {
  const lds_f* la;
  const lds_f* lb;
  const lds_f* lc;
  float* C;
  int m, n, k;
  int lda, ldb, ldc;
  float alpha, beta;
};

// How a block waits for the staging copies before it reads LDS: not at all
// (an earlier block of the same wavefront already did), for this
// wavefront's own copies, or for the whole work-group's copies (barrier).
enum { SYNC_NONE = 0, SYNC_WAVE = 1, SYNC_GROUP = 2 };

__device__ __forceinline__ void staged_sync(int sync) {
  if (sync != SYNC_NONE) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  if (sync == SYNC_GROUP) __syncthreads();
}

// Work-group barrier after the staging copies have landed (executed by the
// first block each wavefront runs on a problem, or in its place).
__device__ __forceinline__ void staged_barrier() { staged_sync(SYNC_GROUP); }

// op(A)(i,k) and op(B)(k,j) inside the staged copies.
template <int TA>
__device__ __forceinline__ float opa(const LdsProb& P, int i, int k) {
  return TA ? P.la[k + i * P.lda] : P.la[i + k * P.lda];
}
template <int TB>
__device__ __forceinline__ float opb(const LdsProb& P, int k, int j) {
  return TB ? P.lb[j + k * P.ldb] : P.lb[k + j * P.ldb];
}

__device__ __forceinline__ float epi_pre(float alpha, float acc, float beta, float c) {
  return beta == 0.0f ? alpha * acc : fmaf(alpha, acc, beta * c);
}

// C(i, j) from the staged copy (0 when C is not read: beta == 0).
__device__ __forceinline__ float cval(const LdsProb& P, int i, int j) {
  return P.lc != nullptr ? P.lc[i + j * P.ldc] : 0.0f;
}

// ---------------------------------------------------------------------------
// Matrix-core scheme from LDS: a TM x TN grid (TM, TN <= 3 given at run time)
// of 16x16 tiles.  Every tile of the grid gets exactly MfmaBlock's sequence of
// v_mfma_f32_16x16x4_f32 (same lane layout, same k order, same zero-filled
// last chunk) and epilogue; tiles outside TM x TN are skipped by wave-uniform
// branches, so one routine serves all nine grid shapes.
template <int TA, int TB>
struct LdsMfma {
  static __device__ __forceinline__ void run(const LdsProb& P, int i0, int j0, int sync, int TM,
                                             int TN) {
    const int l = lane();
    const int r = l & 15, g = l >> 4;
    const rsrc_t rc = rsrc(P.C);
    const uint32_t ldc = (uint32_t)P.ldc;
    staged_sync(sync);
    int ia[3], jb[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      ia[t] = min(i0 + 16 * t + r, P.m - 1);
      jb[t] = min(j0 + 16 * t + r, P.n - 1);
    }
    f4 acc[3][3];
#pragma unroll
    for (int tm = 0; tm < 3; ++tm)
#pragma unroll
      for (int tn = 0; tn < 3; ++tn) acc[tm][tn] = f4{0.f, 0.f, 0.f, 0.f};
    const int nfull = P.k >> 4;
    const int rem = P.k - (nfull << 4);
    const int nchunk = nfull + (rem > 0 ? 1 : 0);
    for (int c = 0; c < nchunk; ++c) {
      const bool tail = c == nfull;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * g + s;
        const bool ok = !tail || kk < rem;
        const int kc = 16 * c + (tail ? min(kk, rem - 1) : kk);
        float a[3], b[3];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
          const float va = opa<TA>(P, ia[t], kc);
          const float vb = opb<TB>(P, kc, jb[t]);
          a[t] = ok ? va : 0.0f;
          b[t] = ok ? vb : 0.0f;
        }
#pragma unroll
        for (int tm = 0; tm < 3; ++tm)
#pragma unroll
          for (int tn = 0; tn < 3; ++tn)
            if (tm < TM && tn < TN)
              acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[tm], b[tn], acc[tm][tn], 0, 0, 0);
      }
    }
    const float alpha = P.alpha, beta = P.beta;
#pragma unroll
    for (int tn = 0; tn < 3; ++tn) {
      const int j = j0 + 16 * tn + r;
      if (tn >= TN || j >= P.n) continue;
#pragma unroll
      for (int tm = 0; tm < 3; ++tm) {
        if (tm >= TM) continue;
        const int ib = i0 + 16 * tm + 4 * g;
        const uint32_t oc = 4 * ((uint32_t)ib + (uint32_t)j * ldc);
        if (ib + 3 < P.m) {
          f4u o;
          o.x = epi_pre(alpha, acc[tm][tn].x, beta, cval(P, ib + 0, j));
          o.y = epi_pre(alpha, acc[tm][tn].y, beta, cval(P, ib + 1, j));
          o.z = epi_pre(alpha, acc[tm][tn].z, beta, cval(P, ib + 2, j));
          o.w = epi_pre(alpha, acc[tm][tn].w, beta, cval(P, ib + 3, j));
          bst4(rc, oc, o);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ib + v < P.m) bst(rc, oc + 4 * v, epi_pre(alpha, acc[tm][tn][v], beta, cval(P, ib + v, j)));
        }
      }
    }
  }
};

// Row strip from LDS with the strip height MR <= 8 given at run time: eight
// FMA chains over k in increasing order (rows past MR repeat row MR-1 and are
// not stored), so each stored element gets exactly RowsBlock's chain.
template <int TA, int TB>
struct LdsRows {
  static __device__ __forceinline__ void run(const LdsProb& P, int i0, int j0, int sync, int MR) {
    const int j = j0 + lane();
    const int jc = min(j, P.n - 1);
    const rsrc_t rc = rsrc(P.C);
    const uint32_t oc = 4 * ((uint32_t)i0 + (uint32_t)j * (uint32_t)P.ldc);
    staged_sync(sync);
    int ri[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) ri[i] = i0 + min(i, MR - 1);
    float acc[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = 0.0f;
    for (int k = 0; k < P.k; ++k) {
      const float b = opb<TB>(P, k, jc);
#pragma unroll
      for (int i = 0; i < 8; ++i) acc[i] = fmaf(opa<TA>(P, ri[i], k), b, acc[i]);
    }
    if (j < P.n) {
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (i < MR) bst(rc, oc + 4 * i, epi_pre(P.alpha, acc[i], P.beta, cval(P, i0 + i, j)));
    }
  }
};

// Column strip from LDS with NR <= 8 given at run time (mirror image).
template <int TA, int TB>
struct LdsCols {
  static __device__ __forceinline__ void run(const LdsProb& P, int i0, int j0, int sync, int NR) {
    const int i = i0 + lane();
    const int ic = min(i, P.m - 1);
    const rsrc_t rc = rsrc(P.C);
    const uint32_t ldc = (uint32_t)P.ldc;
    staged_sync(sync);
    int cj[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) cj[j] = j0 + min(j, NR - 1);
    float acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.0f;
    for (int k = 0; k < P.k; ++k) {
      const float a = opa<TA>(P, ic, k);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[j] = fmaf(a, opb<TB>(P, k, cj[j]), acc[j]);
    }
    if (i < P.m) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < NR)
          bst(rc, 4 * ((uint32_t)i + (uint32_t)(j0 + j) * ldc),
              epi_pre(P.alpha, acc[j], P.beta, cval(P, i, j0 + j)));
    }
  }
};

// K-split block from LDS with MR, NR <= 4 given at run time (4 x 4 chains,
// rows/columns past MR/NR repeat the last one and are not stored; each
// stored element gets exactly KredBlock's sum and butterfly).
template <int TA, int TB>
struct LdsKred {
  static __device__ __forceinline__ void run(const LdsProb& P, int i0, int j0, int sync, int MR,
                                             int NR) {
    const int l = lane();
    const rsrc_t rc = rsrc(P.C);
    const uint32_t ldc = (uint32_t)P.ldc;
    staged_sync(sync);
    int ri[4], cj[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      ri[t] = i0 + min(t, MR - 1);
      cj[t] = j0 + min(t, NR - 1);
    }
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.0f;
    for (int k = l; k < P.k; k += 64) {
      float a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = opa<TA>(P, ri[i], k);
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = opb<TB>(P, k, cj[j]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        float v = acc[i][j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[i][j] = v;
      }
    if (l == 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (i < MR && j < NR)
            bst(rc, 4 * ((uint32_t)(i0 + i) + (uint32_t)(j0 + j) * ldc),
                epi_pre(P.alpha, acc[i][j], P.beta, cval(P, i0 + i, j0 + j)));
    }
  }
};

}  // namespace dev
}  // namespace iaat
