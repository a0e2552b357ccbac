// Wavefront-level block kernels of the generated family (Section IV: one
// size-specialised kernel per block shape and layout).  Each computes one
// block of C = alpha*op(A)*op(B) + beta*C straight from the caller's
// column-major A and B: no pack copy (Section I's motivation), no split of
// K (Section V-A: A and B blocks span all of K), and no per-element bounds
// test inside the K loop.  Rows/columns past the sub-problem edge are read
// from the last valid row/column (clamped addresses) and their results are
// dropped at the store; only the last partial K chunk of the matrix-core
// scheme selects zeros.
//
// op(A)(i,p) = A[i + p*lda] (N) or A[p + i*lda] (T); op(B)(p,j) = B[p + j*ldb]
// (N) or B[j + p*ldb] (T).
//
// Addressing: every operand is a wave-uniform buffer resource whose 64-bit
// base advances along K by scalar adds, plus a 32-bit per-lane byte offset.  Inside a sub-problem
// of at most 80 x 80 the offsets stay below 2^32 while every leading
// dimension is at most kNarrowLd; problems with a larger leading dimension
// take the 64-bit wide_subproblem instead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace iaat {
namespace dev {

typedef float f4 __attribute__((ext_vector_type(4)));
// 16-byte vector with only 4-byte alignment (gfx950 memory accesses accept it).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int64_t kNarrowLd = 1 << 22;

__device__ __forceinline__ int lane() { return (int)(threadIdx.x & 63); }

// Raw buffer access: a wave-uniform resource (base address in SGPRs, no
// range limit, the gfx9-family format word) plus a 32-bit per-lane byte
// offset and a wave-uniform scalar byte offset.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
__device__ __forceinline__ float bld(rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ f4u bld4(rsrc_t r, uint32_t voff, uint32_t soff = 0) {
  const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
  return __builtin_bit_cast(f4u, v);
}
__device__ __forceinline__ void bst(rsrc_t r, uint32_t voff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)voff, 0, 0);
}
__device__ __forceinline__ void bst4(rsrc_t r, uint32_t voff, f4u v) {
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, v), r, (int)voff, 0, 0);
}

// The epilogue of every scheme: C = alpha*acc + beta*C, C unread if beta == 0.
__device__ __forceinline__ float epi(float alpha, float acc, float beta, const float* c) {
  return beta == 0.0f ? alpha * acc : fmaf(alpha, acc, beta * *c);
}
__device__ __forceinline__ void epi_store(rsrc_t rc, uint32_t off, float alpha, float acc,
                                          float beta) {
  bst(rc, off, beta == 0.0f ? alpha * acc : fmaf(alpha, acc, beta * bld(rc, off)));
}

// ---------------------------------------------------------------------------
// Matrix-core scheme: TM x TN grid of 16x16 tiles, v_mfma_f32_16x16x4_f32.
// Operand layout of that instruction: lane l supplies op(A)(row l%16, k-slot
// l/16) and op(B)(k-slot l/16, col l%16); the 16x16 result sits in 4 VGPRs,
// lane l holding rows 4*(l/16)+v (v = 0..3) of column l%16.
// K is consumed in chunks of 16.  Within a chunk, step s (0..3) gives lane
// group g = l/16 the reduction index k = 4g + s, so each lane reads four
// consecutive k of one row/column: one 16-byte load where that run is
// contiguous in memory (op(A) = A^T, op(B) = B), four strided loads otherwise.
// Chunks are double-buffered: the loads of chunk c+1 are in flight while
// chunk c runs on the matrix cores (the ping-pong idea of Section IV-B, where
// one stage computes while the next stage's operands are loaded).
template <int TA, int TB, int TM, int TN>
struct MfmaBlock {
  struct Buf {
    float a[TM][4];
    float b[TN][4];
  };

  static __device__ __forceinline__ void load(Buf& u, rsrc_t ra, rsrc_t rb, const uint32_t (&oa)[TM],
                                              const uint32_t (&ob)[TN], uint32_t lda4,
                                              uint32_t ldb4) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      if (TA) {
        const f4u v = bld4(ra, oa[t]);
        u.a[t][0] = v.x; u.a[t][1] = v.y; u.a[t][2] = v.z; u.a[t][3] = v.w;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) u.a[t][s] = bld(ra, oa[t], s * lda4);
      }
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      if (!TB) {
        const f4u v = bld4(rb, ob[t]);
        u.b[t][0] = v.x; u.b[t][1] = v.y; u.b[t][2] = v.z; u.b[t][3] = v.w;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) u.b[t][s] = bld(rb, ob[t], s * ldb4);
      }
    }
  }

  static __device__ __forceinline__ void mma(f4 (&acc)[TM][TN], const Buf& u) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int tm = 0; tm < TM; ++tm)
#pragma unroll
        for (int tn = 0; tn < TN; ++tn)
          acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(u.a[tm][s], u.b[tn][s],
                                                             acc[tm][tn], 0, 0, 0);
  }

  static __device__ __forceinline__ void run(const Prob& P, int i0, int j0) {
    const int l = lane();
    const int r = l & 15, g = l >> 4;
    const uint32_t lda = (uint32_t)P.lda, ldb = (uint32_t)P.ldb, ldc = (uint32_t)P.ldc;
    const uint32_t lda4 = 4 * lda, ldb4 = 4 * ldb;
    // byte offsets of this lane's op(A) row / op(B) column at k-slot 4g of a
    // chunk, relative to the chunk's base
    uint32_t oa[TM], ob[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const uint32_t i = (uint32_t)min(i0 + 16 * t + r, P.m - 1);
      oa[t] = 4 * (TA ? i * lda + 4 * g : i + 4 * g * lda);
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const uint32_t j = (uint32_t)min(j0 + 16 * t + r, P.n - 1);
      ob[t] = 4 * (TB ? j + 4 * g * ldb : j * ldb + 4 * g);
    }
    // K advance per chunk, in elements, of the uniform bases
    const int64_t da = TA ? 16 : 16 * (int64_t)P.lda, db = TB ? 16 * (int64_t)P.ldb : 16;
    const float* pa = P.A;
    const float* pb = P.B;
    f4 acc[TM][TN];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = f4{0.f, 0.f, 0.f, 0.f};

    const int nfull = P.k >> 4;
    Buf u0, u1;
    if (nfull > 0) {
      // ping-pong: while one buffer feeds the matrix cores, the other is
      // being loaded with the next chunk.  Chunk indices past the last full
      // chunk are clamped to it (a cache hit), so the loads are unconditional.
      const int last = nfull - 1;
      load(u0, rsrc(pa), rsrc(pb), oa, ob, lda4, ldb4);
      for (int c = 0; c < nfull; c += 2) {
        const int c1 = min(c + 1, last), c2 = min(c + 2, last);
        load(u1, rsrc(pa + c1 * da), rsrc(pb + c1 * db), oa, ob, lda4, ldb4);
        __builtin_amdgcn_sched_barrier(0);  // keep the prefetch ahead of the math
        mma(acc, u0);
        if (c + 1 > last) break;
        load(u0, rsrc(pa + c2 * da), rsrc(pb + c2 * db), oa, ob, lda4, ldb4);
        __builtin_amdgcn_sched_barrier(0);
        mma(acc, u1);
      }
      pa += nfull * da;
      pb += nfull * db;
    }
    const int rem = P.k - (nfull << 4);
    if (rem > 0) {
      // pa/pb sit on chunk nfull.  Slot 4g+s reads k = min(4g+s, rem-1)
      // (always inside A and B) and contributes zero past rem.
      const rsrc_t ra = rsrc(pa), rb = rsrc(pb);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * g + s;
        const bool ok = kk < rem;
        const uint32_t kc = (uint32_t)min(kk, rem - 1);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
          const uint32_t o = TA ? oa[tm] - 16 * g + 4 * kc : oa[tm] - 16 * g * lda + kc * lda4;
          const float v = bld(ra, o);
          u0.a[tm][s] = ok ? v : 0.0f;
        }
#pragma unroll
        for (int tn = 0; tn < TN; ++tn) {
          const uint32_t o = TB ? ob[tn] - 16 * g * ldb + kc * ldb4 : ob[tn] - 16 * g + 4 * kc;
          const float v = bld(rb, o);
          u0.b[tn][s] = ok ? v : 0.0f;
        }
      }
      mma(acc, u0);
    }

    // epilogue on the valid part of the block
    const float alpha = P.alpha, beta = P.beta;
    const rsrc_t rc = rsrc(P.C);
#pragma unroll
    for (int tn = 0; tn < TN; ++tn) {
      const int j = j0 + 16 * tn + r;
      if (j >= P.n) continue;
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        const int ib = i0 + 16 * tm + 4 * g;
        const uint32_t oc = 4 * ((uint32_t)ib + (uint32_t)j * ldc);
        if (ib + 3 < P.m) {
          f4u o;
          if (beta == 0.0f) {
            o.x = alpha * acc[tm][tn].x;
            o.y = alpha * acc[tm][tn].y;
            o.z = alpha * acc[tm][tn].z;
            o.w = alpha * acc[tm][tn].w;
          } else {
            const f4u c = bld4(rc, oc);
            o.x = fmaf(alpha, acc[tm][tn].x, beta * c.x);
            o.y = fmaf(alpha, acc[tm][tn].y, beta * c.y);
            o.z = fmaf(alpha, acc[tm][tn].z, beta * c.z);
            o.w = fmaf(alpha, acc[tm][tn].w, beta * c.w);
          }
          bst4(rc, oc, o);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ib + v < P.m) epi_store(rc, oc + 4 * v, alpha, acc[tm][tn][v], beta);
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Row-strip scheme: MR rows x 64 columns, lane l owns column j0 + l and keeps
// MR accumulators; for each k, in increasing order, it multiplies the
// wave-uniform op(A)(i,k) by its own op(B)(k,j) -- the vector x lane-scalar
// FMA of the paper's templates (Table 2) with the lane index as the vector
// element.  Columns past N are clamped for loads and not stored.
template <int TA, int TB, int MR>
struct RowsBlock {
  static __device__ __forceinline__ void run(const Prob& P, int i0, int j0) {
    const int j = j0 + lane();
    const uint32_t jc = (uint32_t)min(j, P.n - 1);
    const uint32_t ldb = (uint32_t)P.ldb, ldb4 = 4 * ldb;
    const int64_t lda = (int64_t)P.lda;
    const uint32_t ob = 4 * (TB ? jc : jc * ldb);
    const float* pa = TA ? P.A + (int64_t)i0 * lda : P.A + i0;
    const float* pb = P.B;
    const int K = P.k;
    float acc[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) acc[i] = 0.0f;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
      float b[4];
      const rsrc_t rb = rsrc(pb);
      if (!TB) {
        const f4u v = bld4(rb, ob);
        b[0] = v.x; b[1] = v.y; b[2] = v.z; b[3] = v.w;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) b[s] = bld(rb, ob, s * ldb4);
      }
      float a[MR][4];
#pragma unroll
      for (int i = 0; i < MR; ++i)
#pragma unroll
        for (int s = 0; s < 4; ++s) a[i][s] = TA ? pa[i * lda + s] : pa[i + s * lda];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < MR; ++i) acc[i] = fmaf(a[i][s], b[s], acc[i]);
      pa += TA ? 4 : 4 * lda;
      pb += TB ? 4 * (int64_t)ldb : 4;
    }
    for (; k < K; ++k) {
      const float b = bld(rsrc(pb), ob);
#pragma unroll
      for (int i = 0; i < MR; ++i) acc[i] = fmaf(TA ? pa[i * lda] : pa[i], b, acc[i]);
      pa += TA ? 1 : lda;
      pb += TB ? (int64_t)ldb : 1;
    }
    if (j < P.n) {
      const rsrc_t rc = rsrc(P.C);
      const uint32_t oc = 4 * ((uint32_t)i0 + (uint32_t)j * (uint32_t)P.ldc);
#pragma unroll
      for (int i = 0; i < MR; ++i) epi_store(rc, oc + 4 * i, P.alpha, acc[i], P.beta);
    }
  }
};

// Column-strip scheme: 64 rows x NR columns, lane l owns row i0 + l; the
// op(B)(k,j) values are wave-uniform.  Mirror image of the row strip.
template <int TA, int TB, int NR>
struct ColsBlock {
  static __device__ __forceinline__ void run(const Prob& P, int i0, int j0) {
    const int i = i0 + lane();
    const uint32_t ic = (uint32_t)min(i, P.m - 1);
    const uint32_t lda = (uint32_t)P.lda, lda4 = 4 * lda;
    const int64_t ldb = (int64_t)P.ldb;
    const uint32_t oa = 4 * (TA ? ic * lda : ic);
    const float* pa = P.A;
    const float* pb = TB ? P.B + j0 : P.B + (int64_t)j0 * ldb;
    const int K = P.k;
    float acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = 0.0f;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
      float a[4];
      const rsrc_t ra = rsrc(pa);
      if (TA) {
        const f4u v = bld4(ra, oa);
        a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = bld(ra, oa, s * lda4);
      }
      float b[NR][4];
#pragma unroll
      for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int s = 0; s < 4; ++s) b[j][s] = TB ? pb[j + s * ldb] : pb[j * ldb + s];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = fmaf(a[s], b[j][s], acc[j]);
      pa += TA ? 4 : 4 * (int64_t)lda;
      pb += TB ? 4 * ldb : 4;
    }
    for (; k < K; ++k) {
      const float a = bld(rsrc(pa), oa);
#pragma unroll
      for (int j = 0; j < NR; ++j) acc[j] = fmaf(a, TB ? pb[j] : pb[j * ldb], acc[j]);
      pa += TA ? 1 : (int64_t)lda;
      pb += TB ? ldb : 1;
    }
    if (i < P.m) {
      const uint32_t ldc = (uint32_t)P.ldc;
      const rsrc_t rc = rsrc(P.C);
#pragma unroll
      for (int j = 0; j < NR; ++j)
        epi_store(rc, 4 * ((uint32_t)i + (uint32_t)(j0 + j) * ldc), P.alpha, acc[j], P.beta);
    }
  }
};

// K-split scheme for tiny blocks: lane l accumulates the products with
// k = l, l + 64, ... for all MR x NR outputs, then a butterfly over the 64
// lanes sums the partial results (cross-lane shuffles); lane 0 stores.
template <int TA, int TB, int MR, int NR>
struct KredBlock {
  static __device__ __forceinline__ void run(const Prob& P, int i0, int j0) {
    const int l = lane();
    const uint32_t lda = (uint32_t)P.lda, ldb = (uint32_t)P.ldb;
    uint32_t oa[MR], ob[NR];
#pragma unroll
    for (int i = 0; i < MR; ++i)
      oa[i] = 4 * (TA ? (uint32_t)l + (uint32_t)(i0 + i) * lda
                      : (uint32_t)(i0 + i) + (uint32_t)l * lda);
#pragma unroll
    for (int j = 0; j < NR; ++j)
      ob[j] = 4 * (TB ? (uint32_t)(j0 + j) + (uint32_t)l * ldb
                      : (uint32_t)l + (uint32_t)(j0 + j) * ldb);
    const int64_t da = TA ? 64 : 64 * (int64_t)P.lda, db = TB ? 64 * (int64_t)P.ldb : 64;
    const float* pa = P.A;
    const float* pb = P.B;
    float acc[MR][NR];
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j) acc[i][j] = 0.0f;
    for (int kb = 0; kb < P.k; kb += 64) {
      if (kb + l < P.k) {
        const rsrc_t ra = rsrc(pa), rb = rsrc(pb);
        float a[MR], b[NR];
#pragma unroll
        for (int i = 0; i < MR; ++i) a[i] = bld(ra, oa[i]);
#pragma unroll
        for (int j = 0; j < NR; ++j) b[j] = bld(rb, ob[j]);
#pragma unroll
        for (int i = 0; i < MR; ++i)
#pragma unroll
          for (int j = 0; j < NR; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
      }
      pa += da;
      pb += db;
    }
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        float v = acc[i][j];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[i][j] = v;
      }
    if (l == 0) {
      const uint32_t ldc = (uint32_t)P.ldc;
      const rsrc_t rc = rsrc(P.C);
#pragma unroll
      for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int i = 0; i < MR; ++i)
          epi_store(rc, 4 * ((uint32_t)(i0 + i) + (uint32_t)(j0 + j) * ldc), P.alpha, acc[i][j],
                    P.beta);
    }
  }
};

// Whole sub-problem with 64-bit addressing, for leading dimensions beyond
// kNarrowLd: lane l computes elements l, l+64, ... (column-major order), each
// as one FMA chain over k in increasing order.
template <int TA, int TB>
__device__ __forceinline__ void wide_subproblem(const Prob& P) {
  const int64_t mn = (int64_t)P.m * P.n;
  for (int64_t e = lane(); e < mn; e += 64) {
    const int64_t i = e % P.m, j = e / P.m;
    float s = 0.0f;
    for (int64_t p = 0; p < P.k; ++p) {
      const float a = TA ? P.A[p + i * P.lda] : P.A[i + p * P.lda];
      const float b = TB ? P.B[j + p * P.ldb] : P.B[p + j * P.ldb];
      s = fmaf(a, b, s);
    }
    float* pc = P.C + i + j * P.ldc;
    *pc = epi(P.alpha, s, P.beta, pc);
  }
}

// Quick return for alpha == 0 or K == 0: C = beta*C (beta == 0 writes zeros
// and does not read C), one wavefront walking the columns.
__device__ __forceinline__ void scale_columns(float* C, int m, int n, int ldc, float beta,
                                              int j_begin, int j_step) {
  for (int j = j_begin; j < n; j += j_step) {
    float* pc = C + (int64_t)j * ldc;
    for (int i = lane(); i < m; i += 64) pc[i] = beta == 0.0f ? 0.0f : beta * pc[i];
  }
}

// Family dispatch.
template <int FAM, int TA, int TB, int P1, int P2>
struct BlockOp;
template <int TA, int TB, int P1, int P2>
struct BlockOp<0, TA, TB, P1, P2> : MfmaBlock<TA, TB, P1, P2> {};
template <int TA, int TB, int P1, int P2>
struct BlockOp<1, TA, TB, P1, P2> : RowsBlock<TA, TB, P1> {};
template <int TA, int TB, int P1, int P2>
struct BlockOp<2, TA, TB, P1, P2> : ColsBlock<TA, TB, P2> {};
template <int TA, int TB, int P1, int P2>
struct BlockOp<3, TA, TB, P1, P2> : KredBlock<TA, TB, P1, P2> {};

}  // namespace dev
}  // namespace iaat
