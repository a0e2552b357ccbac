// The batched FP32 kernel: many uneven problems in one persistent launch.
//
// Work-groups stage batches of problems in LDS and run their kernel
// executing plans (Section V-B) from there; problems too large to stage go
// to a companion kernel that reads them straight from memory.
//
// The staged copies are verbatim: each operand's memory span (A, B, and C
// when beta != 0) is copied with 16-byte memory-to-LDS loads and keeps its
// leading dimension, so element (r, c) of a stored matrix sits at
// la + r + c*ld.  This is the GPU counterpart of the paper's operands
// sitting in cache: no reordering and no extra memory traffic (each element
// crosses HBM once), so not a pack step.
//
// A problem's plan blocks are run as units: compile-time-sized members of
// the generated family or pieces of one (a pair of matrix-core tiles, a
// strip of at most four rows or columns, a K-split row).  Cutting a block
// into pieces never changes an element's arithmetic, and each unit performs
// exactly the operations of its direct-from-memory counterpart in tiles.h,
// in the same order, so a problem gets bitwise the same C here as from
// iaat_gemm.
#include <hip/hip_runtime.h>

#include "direct.h"
#include "iaat_internal.h"
#include "kernels.h"
#include "tiles.h"

namespace iaat {
namespace dev {

typedef __attribute__((address_space(3))) float lds_f;

struct SProb {
  const lds_f* a;
  const lds_f* b;
  const lds_f* c;  // staged C, or null: C is read from memory (when beta != 0)
  float* C;
  int m, n, k;
  int lda, ldb, ldc;  // lda, ldb: staged; ldc: memory
  int ldcs;           // staged ldc
  float alpha, beta;
};

// C(i, j) for the epilogue: from memory (CMEM), else the staged copy, or 0
// when beta == 0.  The compute loop inlines only the CMEM = false forms:
// a memory load there would make the compiler wait on the vector-memory
// counter, which on this architecture also counts the wavefront's earlier
// C stores.
template <bool CMEM>
__device__ __forceinline__ float c_at(const SProb& P, rsrc_t rc, int i, int j) {
  if (P.beta == 0.0f) return 0.0f;
  if (CMEM) return bld(rc, 4 * ((uint32_t)i + (uint32_t)j * (uint32_t)P.ldc));
  return P.c[i + j * P.ldcs];
}

template <int TA>
__device__ __forceinline__ float sa(const SProb& P, int i, int k) {
  return TA ? P.a[k + i * P.lda] : P.a[i + k * P.lda];
}
template <int TB>
__device__ __forceinline__ float sb(const SProb& P, int k, int j) {
  return TB ? P.b[j + k * P.ldb] : P.b[k + j * P.ldb];
}
// Four consecutive staged floats.  The staged copies keep the operands'
// memory alignment, so these are four 4-byte reads.
__device__ __forceinline__ f4 ld4(const lds_f* p) { return f4{p[0], p[1], p[2], p[3]}; }

// The lane index, read afresh in every unit: a volatile read cannot be
// hoisted out of the compute loop, so the lane-derived values of the many
// inlined units are not all kept live across it.
__device__ __forceinline__ int lane_u() {
  int v;
  asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
  return v;
}

__device__ __forceinline__ float epi_c(float alpha, float acc, float beta, float c) {
  return beta == 0.0f ? alpha * acc : fmaf(alpha, acc, beta * c);
}

// TM x TN (<= 2 x 2) tiles of 16 x 16 with v_mfma_f32_16x16x4_f32, the
// operation sequence of MfmaBlock: chunks of 16 k, step s of a chunk gives
// lane group g = l/16 the reduction index 4g + s; the last partial chunk
// reads k = min(4g + s, rem - 1) and contributes zero past rem.
template <int TA, int TB, int TM, int TN, bool CMEM>
struct StagedMfma {
  static __device__ __forceinline__ void run(const SProb& P, int i0, int j0) {
    const int l = lane_u();
    const int r = l & 15, g = l >> 4;
    const rsrc_t rc = rsrc(P.C);
    const uint32_t ldc = (uint32_t)P.ldc;
    const float alpha = P.alpha, beta = P.beta;
    // C first, so its memory latency overlaps the K loop
    f4 cv[TM][TN];
#pragma unroll
    for (int tn = 0; tn < TN; ++tn)
#pragma unroll
      for (int tm = 0; tm < TM; ++tm) {
        cv[tm][tn] = f4{0.f, 0.f, 0.f, 0.f};
        const int j = j0 + 16 * tn + r, ib = i0 + 16 * tm + 4 * g;
        if (!CMEM || beta == 0.0f || j >= P.n) continue;
        const uint32_t oc = 4 * ((uint32_t)ib + (uint32_t)j * ldc);
        if (ib + 3 < P.m) {
          const f4u c = bld4(rc, oc);
          cv[tm][tn] = f4{c.x, c.y, c.z, c.w};
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ib + v < P.m) cv[tm][tn][v] = bld(rc, oc + 4 * v);
        }
      }
    // per-lane element offsets of this lane's op(A) row / op(B) column at
    // k-slot 4g of chunk 0
    int oa[TM], ob[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      const int i = min(i0 + 16 * t + r, P.m - 1);
      oa[t] = TA ? i * P.lda + 4 * g : i + 4 * g * P.lda;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const int j = min(j0 + 16 * t + r, P.n - 1);
      ob[t] = TB ? j + 4 * g * P.ldb : j * P.ldb + 4 * g;
    }
    const int da = TA ? 16 : 16 * P.lda, db = TB ? 16 * P.ldb : 16;  // per chunk
    f4 acc[TM][TN];
#pragma unroll
    for (int tm = 0; tm < TM; ++tm)
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) acc[tm][tn] = f4{0.f, 0.f, 0.f, 0.f};
    const int nfull = P.k >> 4;
    const lds_f* pa = P.a;
    const lds_f* pb = P.b;
    // Chunks are double-buffered in registers: the fragments of chunk c+1
    // are read from LDS while chunk c's four steps run on the matrix core.
    struct Frag {
      f4 a[TM], b[TN];
    };
    auto load = [&](Frag& f, const lds_f* qa, const lds_f* qb) {
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        if (TA) {
          f.a[t] = ld4(qa + oa[t]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) f.a[t][s] = qa[oa[t] + s * P.lda];
        }
      }
#pragma unroll
      for (int t = 0; t < TN; ++t) {
        if (!TB) {
          f.b[t] = ld4(qb + ob[t]);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) f.b[t][s] = qb[ob[t] + s * P.ldb];
        }
      }
    };
    auto mma = [&](const Frag& f) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn)
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(f.a[tm][s], f.b[tn][s], acc[tm][tn], 0, 0, 0);
    };
    if (nfull > 0) {
      Frag f0, f1;
      load(f0, pa, pb);
      for (int c = 0; c < nfull; c += 2) {
        if (c + 1 < nfull) load(f1, pa + da, pb + db);
        __builtin_amdgcn_sched_barrier(0);
        mma(f0);
        if (c + 1 >= nfull) {
          pa += da;
          pb += db;
          break;
        }
        if (c + 2 < nfull) load(f0, pa + 2 * da, pb + 2 * db);
        __builtin_amdgcn_sched_barrier(0);
        mma(f1);
        pa += 2 * da;
        pb += 2 * db;
      }
    }
    const int rem = P.k - (nfull << 4);
    if (rem > 0) {
      f4 va[TM], vb[TN];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = 4 * g + s;
        const bool ok = kk < rem;
        const int kc = min(kk, rem - 1);
#pragma unroll
        for (int t = 0; t < TM; ++t) {
          const float v = TA ? pa[oa[t] - 4 * g + kc] : pa[oa[t] - 4 * g * P.lda + kc * P.lda];
          va[t][s] = ok ? v : 0.0f;
        }
#pragma unroll
        for (int t = 0; t < TN; ++t) {
          const float v = TB ? pb[ob[t] - 4 * g * P.ldb + kc * P.ldb] : pb[ob[t] - 4 * g + kc];
          vb[t][s] = ok ? v : 0.0f;
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int tm = 0; tm < TM; ++tm)
#pragma unroll
          for (int tn = 0; tn < TN; ++tn)
            acc[tm][tn] = __builtin_amdgcn_mfma_f32_16x16x4f32(va[tm][s], vb[tn][s], acc[tm][tn], 0, 0, 0);
    }
    if (!CMEM && beta != 0.0f) {  // staged C
#pragma unroll
      for (int tn = 0; tn < TN; ++tn) {
        const int j = min(j0 + 16 * tn + r, P.n - 1);
#pragma unroll
        for (int tm = 0; tm < TM; ++tm) {
          const int ib = i0 + 16 * tm + 4 * g;
          const lds_f* pc = P.c + j * P.ldcs;
          if (ib + 3 < P.m && (ib & 3) == 0) {
            cv[tm][tn] = ld4(pc + ib);
          } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) cv[tm][tn][v] = pc[min(ib + v, P.m - 1)];
          }
        }
      }
    }
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
          o.x = epi_c(alpha, acc[tm][tn].x, beta, cv[tm][tn].x);
          o.y = epi_c(alpha, acc[tm][tn].y, beta, cv[tm][tn].y);
          o.z = epi_c(alpha, acc[tm][tn].z, beta, cv[tm][tn].z);
          o.w = epi_c(alpha, acc[tm][tn].w, beta, cv[tm][tn].w);
          bst4(rc, oc, o);
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (ib + v < P.m) bst(rc, oc + 4 * v, epi_c(alpha, acc[tm][tn][v], beta, cv[tm][tn][v]));
        }
      }
    }
  }
};

// MR rows x 64 columns, lane = column (RowsBlock's operation sequence: FMA
// chains over k in increasing order, four k at a time, then the rest).
template <int TA, int TB, int MR, bool CMEM>
struct StagedRows {
  static __device__ __forceinline__ void run(const SProb& P, int i0, int j0) {
    const int j = j0 + lane_u();
    const int jc = min(j, P.n - 1);
    const rsrc_t rc = rsrc(P.C);
    const uint32_t oc = 4 * ((uint32_t)i0 + (uint32_t)j * (uint32_t)P.ldc);
    const bool st = j < P.n;
    float cv[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) cv[i] = (CMEM && st) ? c_at<true>(P, rc, i0 + i, j) : 0.0f;
    float acc[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) acc[i] = 0.0f;
    const int K = P.k;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
      f4 b;
      if (!TB) {
        b = ld4(P.b + jc * P.ldb + k);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) b[s] = P.b[jc + (k + s) * P.ldb];
      }
      f4 a[MR];
#pragma unroll
      for (int i = 0; i < MR; ++i) {
        if (TA) {
          a[i] = ld4(P.a + (i0 + i) * P.lda + k);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) a[i][s] = P.a[(i0 + i) + (k + s) * P.lda];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int i = 0; i < MR; ++i) acc[i] = fmaf(a[i][s], b[s], acc[i]);
    }
    for (; k < K; ++k) {
      const float b = sb<TB>(P, k, jc);
#pragma unroll
      for (int i = 0; i < MR; ++i) acc[i] = fmaf(sa<TA>(P, i0 + i, k), b, acc[i]);
    }
    if (!CMEM) {
#pragma unroll
      for (int i = 0; i < MR; ++i) cv[i] = c_at<false>(P, rc, i0 + i, jc);
    }
    if (st) {
#pragma unroll
      for (int i = 0; i < MR; ++i) bst(rc, oc + 4 * i, epi_c(P.alpha, acc[i], P.beta, cv[i]));
    }
  }
};

// 64 rows x NR columns, lane = row (mirror image of the row strip).
template <int TA, int TB, int NR, bool CMEM>
struct StagedCols {
  static __device__ __forceinline__ void run(const SProb& P, int i0, int j0) {
    const int i = i0 + lane_u();
    const int ic = min(i, P.m - 1);
    const rsrc_t rc = rsrc(P.C);
    const uint32_t ldc = (uint32_t)P.ldc;
    const bool st = i < P.m;
    float cv[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) cv[j] = (CMEM && st) ? c_at<true>(P, rc, i, j0 + j) : 0.0f;
    float acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = 0.0f;
    const int K = P.k;
    int k = 0;
    for (; k + 4 <= K; k += 4) {
      f4 a;
      if (TA) {
        a = ld4(P.a + ic * P.lda + k);
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) a[s] = P.a[ic + (k + s) * P.lda];
      }
      f4 b[NR];
#pragma unroll
      for (int j = 0; j < NR; ++j) {
        if (!TB) {
          b[j] = ld4(P.b + (j0 + j) * P.ldb + k);
        } else {
#pragma unroll
          for (int s = 0; s < 4; ++s) b[j][s] = P.b[(j0 + j) + (k + s) * P.ldb];
        }
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc[j] = fmaf(a[s], b[j][s], acc[j]);
    }
    for (; k < K; ++k) {
      const float a = sa<TA>(P, ic, k);
#pragma unroll
      for (int j = 0; j < NR; ++j) acc[j] = fmaf(a, sb<TB>(P, k, j0 + j), acc[j]);
    }
    if (!CMEM) {
#pragma unroll
      for (int j = 0; j < NR; ++j) cv[j] = c_at<false>(P, rc, ic, j0 + j);
    }
    if (st) {
#pragma unroll
      for (int j = 0; j < NR; ++j)
        bst(rc, 4 * ((uint32_t)i + (uint32_t)(j0 + j) * ldc), epi_c(P.alpha, acc[j], P.beta, cv[j]));
    }
  }
};

// MR x NR (<= 4 x 4) block, K split over the lanes: lane l sums k = l,
// l + 64, ...; a butterfly adds the 64 partial sums; lane 0 stores
// (KredBlock's operation sequence).
template <int TA, int TB, int MR, int NR, bool CMEM>
struct StagedKred {
  static __device__ __forceinline__ void run(const SProb& P, int i0, int j0) {
    const int l = lane_u();
    float acc[MR][NR];
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j) acc[i][j] = 0.0f;
    for (int kb = 0; kb < P.k; kb += 64) {
      const int k = kb + l;
      if (k < P.k) {
        float a[MR], b[NR];
#pragma unroll
        for (int i = 0; i < MR; ++i) a[i] = sa<TA>(P, i0 + i, k);
#pragma unroll
        for (int j = 0; j < NR; ++j) b[j] = sb<TB>(P, k, j0 + j);
#pragma unroll
        for (int i = 0; i < MR; ++i)
#pragma unroll
          for (int j = 0; j < NR; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
      }
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
          bst(rc, 4 * ((uint32_t)(i0 + i) + (uint32_t)(j0 + j) * ldc),
              epi_c(P.alpha, acc[i][j], P.beta, c_at<CMEM>(P, rc, i0 + i, j0 + j)));
    }
  }
};

// The units the batched kernel runs.  Each is a compile-time-sized member of
// the family or a piece of one; cutting a block into pieces never changes an
// element's arithmetic (a matrix-core tile, a row's or a column's FMA chain,
// one output's K-split sum are each computed whole by one unit), so a
// problem's C stays bitwise that of the per-call kernel.
//   U_TILE            one 16 x 16 matrix-core tile
//   U_TILE2           two horizontally adjacent tiles (16 x 32)
//   U_ROWS + r - 1    row strip, r = 1..4 rows x 64 columns
//   U_COLS + c - 1    column strip, 64 rows x c = 1..4 columns
//   U_KRED + c - 1    K-split block of 1 row x c = 1..4 columns
// Few, small units keep the compute loop's code within the instruction
// cache.
// Unit ids, from the generated list (IAAT_FOR_EACH_STAGED_UNIT).
enum {
  U_TILE = IAAT_U_TILE,
  U_TILE2 = IAAT_U_TILE2,
  U_ROWS = IAAT_U_ROWS,
  U_COLS = IAAT_U_COLS,
  U_KRED = IAAT_U_KRED,
  U_COUNT = IAAT_NUM_STAGED_UNITS
};

// The staged routine of a generated unit (family, p1, p2).
template <int FAM, int TA, int TB, int P1, int P2, bool CMEM>
struct StagedUnit;
template <int TA, int TB, int P1, int P2, bool CMEM>
struct StagedUnit<0, TA, TB, P1, P2, CMEM> : StagedMfma<TA, TB, P1, P2, CMEM> {};
template <int TA, int TB, int P1, int P2, bool CMEM>
struct StagedUnit<1, TA, TB, P1, P2, CMEM> : StagedRows<TA, TB, P1, CMEM> {};
template <int TA, int TB, int P1, int P2, bool CMEM>
struct StagedUnit<2, TA, TB, P1, P2, CMEM> : StagedCols<TA, TB, P2, CMEM> {};
template <int TA, int TB, int P1, int P2, bool CMEM>
struct StagedUnit<3, TA, TB, P1, P2, CMEM> : StagedKred<TA, TB, P1, P2, CMEM> {};

template <int TA, int TB, bool CMEM>
__device__ __forceinline__ void unit_body(int u, const SProb& P, int i0, int j0) {
  switch (u) {
#define IAAT_UNIT_CASE(uid, fam, p1, p2)                      \
  case uid:                                                  \
    StagedUnit<fam, TA, TB, p1, p2, CMEM>::run(P, i0, j0); \
    break;
    IAAT_FOR_EACH_STAGED_UNIT(IAAT_UNIT_CASE)
#undef IAAT_UNIT_CASE
    default:
      break;
  }
}

// C is always staged when it is read (beta != 0), so the units never load
// from memory.
template <int TA, int TB>
__device__ __forceinline__ void run_unit(int u, const SProb& P, int i0, int j0) {
  unit_body<TA, TB, false>(u, P, i0, j0);
}


// ---- batched kernel: staged batches --------------------------------------
//
// Work-groups of eight wavefronts, two per CU (each owns half of the LDS,
// so while one work-group waits for its copies the other computes).
// Problems go to work-groups in windows of consecutive problems: first one
// window of s0 problems per work-group, in order; then, with a ticket
// counter, windows of shrinking size (guided self-scheduling: about the
// remaining problems over twice the grid, 4..16) to whichever work-group
// asks next, balancing the uneven work; without one, window w of size s0
// to work-group w mod G.  Wavefront 0 packs a batch -- as many of the
// work-group's next problems as fit into its staging buffer, one problem
// per lane -- into one of two table sets.  The next window is fetched in
// three dependent steps (claim, descriptors, plans), one step per batch,
// so each step's latency hides behind a batch's copies.  Every
// wavefront copies its share of the batch's A, B and (when beta != 0) C
// spans verbatim into LDS with memory-to-LDS loads; after one wait,
// wavefronts 1..7 run the batch's units round-robin (longest first) from
// LDS, storing C, while wavefront 0 packs the next batch.  A barrier closes
// the iteration because the buffer is refilled.  Problems that do not fit the buffer are
// left to vbatched_direct_kernel; quick returns and status codes are handled
// here.

constexpr int kStage = 19312;        // floats of staging per work-group (>= one 80x80x80 problem)
constexpr int kMaxBatch = 16;        // problems per batch
constexpr int kMaxUnits = 128;       // units per batch
constexpr int kWaves = 8;
constexpr int kWin = 16;             // most problems per window (one per lane)

struct BatchProb {  // 64 bytes
  float* C;
  int la, lb, lc;  // float offsets into the staging buffer; lc < 0: C not staged
  int m, n, k, lda, ldb, ldc;
  float alpha, beta;
  int trans;
  int pad[2];
};

// One span copy of a batch: 16-byte-aligned source, staging offset (floats),
// 16-byte units.
struct CopyJob {
  const float* src;
  int dst, n4;
};

__shared__ __attribute__((aligned(16))) float g_stage[kStage];
// Batch tables, double-buffered: wavefront 0 packs batch i+1 while batch i
// is computed.
__shared__ __attribute__((aligned(16))) BatchProb g_bprob[2][kMaxBatch];
// i0 | j0 << 8 | unit << 16 | problem slot << 24; the longer units (all but
// single tiles) from the front, the single tiles from the back, so the
// compute wavefronts take the longest first and the batch ends evenly
__shared__ uint32_t g_bunit[2][kMaxUnits];
__shared__ CopyJob g_copy[2][3 * kMaxBatch];
__shared__ int g_bhead[2][4];  // problems, units, long units, more-to-come

// Staged size of one problem: A, B and (beta != 0) C spans, each widened to
// whole 16-byte units around it.
struct PcGeom {
  int a_sh, b_sh, c_sh;
  int a_n4, b_n4, c_n4;
  bool fits;
};

__device__ __forceinline__ PcGeom pc_geom(const Prob& P, int ta, int tb) {
  PcGeom g;
  const int64_t span_a = (int64_t)P.lda * ((ta ? P.m : P.k) - 1) + (ta ? P.k : P.m);
  const int64_t span_b = (int64_t)P.ldb * ((tb ? P.k : P.n) - 1) + (tb ? P.n : P.k);
  const int64_t span_c = P.beta != 0.0f ? (int64_t)P.ldc * (P.n - 1) + P.m : 0;
  g.a_sh = (int)(((uintptr_t)P.A & 15) >> 2);
  g.b_sh = (int)(((uintptr_t)P.B & 15) >> 2);
  g.c_sh = (int)(((uintptr_t)P.C & 15) >> 2);
  const int64_t a_n4 = (g.a_sh + span_a + 3) >> 2, b_n4 = (g.b_sh + span_b + 3) >> 2;
  const int64_t c_n4 = span_c > 0 ? (g.c_sh + span_c + 3) >> 2 : 0;
  g.fits = P.m <= kSuper && P.n <= kSuper && narrow(P) && 4 * (a_n4 + b_n4 + c_n4) <= kStage;
  g.a_n4 = g.fits ? (int)a_n4 : 0;
  g.b_n4 = g.fits ? (int)b_n4 : 0;
  g.c_n4 = g.fits ? (int)c_n4 : 0;
  return g;
}

// One 16-byte memory-to-LDS load: this lane's 16 bytes land at `base` + 16 *
// lane (`base` is the same for the whole wavefront).
__device__ __forceinline__ void copy16_lds(const float* g16, lds_f* base) {
  typedef __attribute__((address_space(1))) const void gvoid;
  typedef __attribute__((address_space(3))) void lvoid;
  __builtin_amdgcn_global_load_lds((gvoid*)g16, (lvoid*)base, 16, 0, 0);
}

__device__ __forceinline__ int rdl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t rdl(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ float rdlf(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// A window's descriptors (lane l < n holds problem base + l) and their plans.
struct DescWindow {
  uint32_t w[16];   // the iaat_problem words
  uint32_t pl[16];  // the plan entry: block count, blocks
};

__device__ __forceinline__ void window_load(DescWindow& W, const VbArgs& a, int64_t base, int n) {
  const int64_t q = base + min(lane() & (kWin - 1), n - 1);  // lanes >= n repeat the last one
  const u4* src = reinterpret_cast<const u4*>(a.probs + q);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const u4 v = src[i];
    W.w[4 * i + 0] = v.x;
    W.w[4 * i + 1] = v.y;
    W.w[4 * i + 2] = v.z;
    W.w[4 * i + 3] = v.w;
  }
}

__device__ __forceinline__ void window_load_plan(DescWindow& W, const PlanEntry* table) {
  const int trans = (int)W.w[6];
  const int m = min(max((int)W.w[7], 1), kSuper), n = min(max((int)W.w[8], 1), kSuper);
  const u4* e = reinterpret_cast<const u4*>(table + plan_index(trans & 3, m, n));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const u4 v = e[i];
    W.pl[4 * i + 0] = v.x;
    W.pl[4 * i + 1] = v.y;
    W.pl[4 * i + 2] = v.z;
    W.pl[4 * i + 3] = v.w;
  }
}

// The units of one plan block: matrix-core grids as pairs of tiles along
// each row, a row's odd tile alone (tiles wholly outside the problem
// dropped), strips in pieces of at most 4 rows or columns, K-split blocks
// row by row.  block_units counts them in closed form -- `nl` long units
// (all but single tiles) and `ns` single tiles -- and emit_block writes
// them, long ones at ascending indices from `el`, single tiles at
// descending indices from `es`; both follow the same decomposition, so a
// block always writes exactly the units counted for it.
__device__ __forceinline__ void block_units(uint32_t w, int m, int n, int& nl, int& ns) {
  const int kid = blk_kid(w), i0 = blk_i0(w), j0 = blk_j0(w);
  nl = 0;
  ns = 0;
  if (kid < 9) {
    const int tm = kid / 3 + 1, tn = kid % 3 + 1;
    const int ri = min(tm, max(0, (m - i0 + 15) >> 4));  // tile rows inside the problem
    const int ci = min(tn, max(0, (n - j0 + 15) >> 4));  // tile columns inside
    nl = ri * (ci >> 1);
    ns = ri * (ci & 1);
  } else if (kid < 17) {
    nl = (kid - 8 + 3) >> 2;
  } else if (kid < 25) {
    nl = (kid - 16 + 3) >> 2;
  } else {
    nl = (kid - 25) / 4 + 1;
  }
}

__device__ __forceinline__ void emit_block(uint32_t* units, uint32_t w, int m, int n, uint32_t tag,
                                           int el, int es) {
  const int kid = blk_kid(w), i0 = blk_i0(w), j0 = blk_j0(w);
  auto put = [&](int idx, int u, int i, int j) {
    units[idx] = (uint32_t)i | ((uint32_t)j << 8) | ((uint32_t)u << 16) | tag;
  };
  if (kid < 9) {
    const int tm = kid / 3 + 1, tn = kid % 3 + 1;
    const int ri = min(tm, max(0, (m - i0 + 15) >> 4));
    const int ci = min(tn, max(0, (n - j0 + 15) >> 4));
    const int pairs = ci >> 1;
    for (int ti = 0; ti < ri; ++ti) {
      for (int c = 0; c < pairs; ++c) put(el++, U_TILE2, i0 + 16 * ti, j0 + 32 * c);
      if (ci & 1) put(es--, U_TILE, i0 + 16 * ti, j0 + 32 * pairs);
    }
  } else if (kid < 17) {
    const int mr = kid - 8;
    for (int r = 0; r < mr; r += 4) put(el++, U_ROWS + min(4, mr - r) - 1, i0 + r, j0);
  } else if (kid < 25) {
    const int nr = kid - 16;
    for (int c = 0; c < nr; c += 4) put(el++, U_COLS + min(4, nr - c) - 1, i0, j0 + c);
  } else {
    const int mr = (kid - 25) / 4 + 1, nr = (kid - 25) % 4 + 1;
    for (int r = 0; r < mr; ++r) put(el++, U_KRED + nr - 1, i0 + r, j0);
  }
}

// The problem held by this lane / by lane `l` of a window.
__device__ __forceinline__ Prob lane_prob(const DescWindow& W) {
  const uint64_t A = ((uint64_t)W.w[1] << 32) | W.w[0];
  const uint64_t B = ((uint64_t)W.w[3] << 32) | W.w[2];
  const uint64_t C = ((uint64_t)W.w[5] << 32) | W.w[4];
  return Prob{(const float*)A, (const float*)B, (float*)C, (int)W.w[7], (int)W.w[8], (int)W.w[9],
              (int)W.w[10], (int)W.w[11], (int)W.w[12],
              __builtin_bit_cast(float, W.w[13]) * __builtin_bit_cast(float, W.w[15]),
              __builtin_bit_cast(float, W.w[14])};
}

__device__ __forceinline__ Prob lane_prob_of(const DescWindow& W, int l) {
  const uint64_t A = ((uint64_t)rdl(W.w[1], l) << 32) | rdl(W.w[0], l);
  const uint64_t B = ((uint64_t)rdl(W.w[3], l) << 32) | rdl(W.w[2], l);
  const uint64_t C = ((uint64_t)rdl(W.w[5], l) << 32) | rdl(W.w[4], l);
  return Prob{(const float*)A, (const float*)B, (float*)C, (int)rdl(W.w[7], l), (int)rdl(W.w[8], l),
              (int)rdl(W.w[9], l), (int)rdl(W.w[10], l), (int)rdl(W.w[11], l),
              (int)rdl(W.w[12], l),
              __builtin_bit_cast(float, rdl(W.w[13], l)) * __builtin_bit_cast(float, rdl(W.w[15], l)),
              __builtin_bit_cast(float, rdl(W.w[14], l))};
}

// Per-lane view of one problem of the current window (lane l < kWin holds
// problem win*kWin + l): its class and, when it is staged, its copy jobs.
enum { CLS_NONE = 0, CLS_QUICK = 1, CLS_STAGE = 2, CLS_DIRECT = 3 };

struct LaneProb {
  int cls, st, need, nbp, nlong;  // nbp units, nlong of them not single tiles
};

__device__ __forceinline__ LaneProb classify(const DescWindow& W, bool valid_lane) {
  LaneProb r{};
  const Prob P = lane_prob(W);
  const int trans = (int)W.w[6];
  r.st = validate(trans, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.A, P.B, P.C);
  if (!valid_lane || r.st != 0 || P.m == 0 || P.n == 0) {
    r.cls = CLS_NONE;
  } else if (P.alpha == 0.0f || P.k == 0) {
    r.cls = CLS_QUICK;
  } else {
    const PcGeom g = pc_geom(P, trans & 1, trans >> 1);
    r.cls = g.fits ? CLS_STAGE : CLS_DIRECT;
    r.need = g.fits ? 4 * (g.a_n4 + g.b_n4 + g.c_n4) : 0;
    int nu = 0, nl = 0;
    if (g.fits) {
#pragma unroll
      for (int b = 0; b < kMaxBlocks; ++b) {
        if (b < (int)W.pl[0]) {
          int bl, bs;
          block_units(W.pl[1 + b], P.m, P.n, bl, bs);
          nu += bl + bs;
          nl += bl;
        }
      }
    }
    r.nbp = nu;
    r.nlong = nl;
  }
  return r;
}

// Inclusive prefix sum over the first kWin = 16 lanes (one DPP row: each
// step adds the value `off` lanes down the row, 0 past its start).
__device__ __forceinline__ int scan16(int v) {
  static_assert(kWin == 16, "one DPP row");
  v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
  v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
  return v;
}

// The packer's window stream.  `cur` is the window being packed (lanes
// i.. of it still to take); `nxt` the one after it, fetched a step per batch:
// hop 1 claims it (the ticket's old value arrives with the next wait),
// hop 2 loads its descriptors, hop 3 its plans.
struct Windows {
  DescWindow cur, nxt;
  LaneProb lp;         // per-lane class of cur's problems
  int64_t base0;       // cur: problems base0 .. base0 + n0 - 1
  int n0, i;
  int64_t base1;       // nxt
  int n1, s1;          // nxt's size; the size asked for at the claim
  int hop;             // steps of nxt done (3: ready)
  bool end;            // no window after cur
  uint32_t tk;         // lane 0: the ticket's value before the claim
  uint32_t t_last;     // the last ticket value seen (a progress estimate)
  int64_t sbase;       // without a ticket: the last static window
};

struct WinShape {
  int64_t count, G, s0;
};

__device__ __forceinline__ WinShape win_shape(const VbArgs& a) {
  WinShape z;
  z.count = a.count;
  z.G = gridDim.x;
  z.s0 = min<int64_t>(kWin, max<int64_t>(1, a.count / (2 * z.G)));
  return z;
}

// One step of fetching nxt (each needs the previous step's loads).
__device__ __forceinline__ void win_step(Windows& S, const VbArgs& a, const WinShape& z) {
  if (S.end) return;
  if (S.hop == 0) {  // claim
    if (a.ticket != nullptr) {
      const int64_t rem = z.count - (z.G * z.s0 + (int64_t)S.t_last);
      S.s1 = (int)min<int64_t>(kWin, max<int64_t>(4, rem / (2 * z.G)));
      if (lane() == 0) S.tk = atomicAdd(a.ticket, (uint32_t)S.s1);
    }
    S.hop = 1;
  } else if (S.hop == 1) {  // descriptors
    int64_t base;
    if (a.ticket != nullptr) {
      S.t_last = (uint32_t)__builtin_amdgcn_readfirstlane((int)S.tk);
      base = z.G * z.s0 + (int64_t)S.t_last;
    } else {
      S.sbase += z.G * z.s0;
      base = S.sbase;
      S.s1 = (int)z.s0;
    }
    if (base >= z.count) {
      S.end = true;
      return;
    }
    S.base1 = base;
    S.n1 = (int)min<int64_t>(S.s1, z.count - base);
    window_load(S.nxt, a, base, S.n1);
    S.hop = 2;
  } else if (S.hop == 2) {  // plans
    window_load_plan(S.nxt, a.table);
    S.hop = 3;
  }
}

// cur := nxt (finishing its fetch if a window went faster than three
// batches), classified, and the claim of the one after it.  False at the end.
__device__ __forceinline__ bool win_advance(Windows& S, const VbArgs& a, const WinShape& z) {
  while (!S.end && S.hop < 3) win_step(S, a, z);
  if (S.end) return false;
  S.cur = S.nxt;
  S.base0 = S.base1;
  S.n0 = S.n1;
  S.i = 0;
  S.lp = classify(S.cur, lane() < S.n0);
  S.hop = 0;
  win_step(S, a, z);
  return true;
}

__device__ __forceinline__ uint32_t bperm(int src_lane, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_ds_bpermute(src_lane << 2, (int)v);
}

// Writes the units of the taken staged problems of the current window:
// long units of a problem from index `el` up, its single tiles from `es`
// down (per-lane values of the problem's lane).  Lane-per-block: four
// problems a round, lane 16q + b holding block b of the round's q-th
// problem (its plan words gathered from the problem's lane), with the
// block's offsets inside its problem from a 16-lane prefix sum.
__device__ __forceinline__ void emit_units(const Windows& S, const LaneProb& LP, bool take, int tb,
                                           int slot, int el, int es) {
  const int l = lane();
  uint32_t sm = (uint32_t)__ballot(take && LP.cls == CLS_STAGE) & 0xffffu;
  const uint32_t tag = (uint32_t)slot << 24;
  const int q = l >> 4, b = l & 15;
  while (sm) {
    // the round's problems: lanes 16q.. take the q-th next set lane of sm
    uint32_t v = sm;
#pragma unroll
    for (int r = 0; r < 3; ++r)
      if (q > r) v &= v - 1;
    const int p = v ? __builtin_ctz(v) : -1;
#pragma unroll
    for (int r = 0; r < 4; ++r) sm &= sm - 1;
    const int src = p < 0 ? 0 : p;
    uint32_t w = 0;
#pragma unroll
    for (int j = 1; j < 16; ++j) {
      const uint32_t x = bperm(src, S.cur.pl[j]);
      if (b == j - 1) w = x;
    }
    const int nblk = (int)bperm(src, S.cur.pl[0]);
    const int m = (int)bperm(src, S.cur.w[7]), n = (int)bperm(src, S.cur.w[8]);
    const int pel = (int)bperm(src, (uint32_t)el), pes = (int)bperm(src, (uint32_t)es);
    const uint32_t ptag = bperm(src, tag);
    const bool valid = p >= 0 && b < nblk;
    int bl = 0, bs = 0;
    if (valid) block_units(w, m, n, bl, bs);
    const int ol = scan16(bl) - bl, os = scan16(bs) - bs;  // earlier blocks of the problem
    if (valid) emit_block(g_bunit[tb], w, m, n, ptag, pel + ol, pes - os);
  }
}

// Wavefront 0 packs the next batch: problems of this work-group's windows,
// in order, while they fit.  All bookkeeping is per lane (one problem per
// lane) plus prefix sums, then every taken lane writes its own table
// entries; so the cost per batch does not grow with the number of problems.
__device__ __forceinline__ void pack_batch(const VbArgs& a, const WinShape& z, Windows& S, int tb) {
  const int l = lane();
  int used = 0, np = 0, nb = 0, nlong = 0;
  bool more = true;
  win_step(S, a, z);  // one fetch step per batch
  for (;;) {
    if (S.i == S.n0 && !win_advance(S, a, z)) {
      more = false;
      break;
    }
    const int i = S.i;
    const LaneProb& LP = S.lp;
    // candidates: lanes >= i that are staged
    const bool cand = l >= i && LP.cls == CLS_STAGE;
    const int c_need = scan16(cand ? LP.need : 0);
    const int c_blk = scan16(cand ? LP.nbp : 0);
    const int c_long = scan16(cand ? LP.nlong : 0);
    const int c_cnt = scan16(cand ? 1 : 0);
    const bool fits = used + c_need <= kStage && nb + c_blk <= kMaxUnits && np + c_cnt <= kMaxBatch;
    // the first staged lane that does not fit ends this batch
    const uint64_t stop = __ballot(cand && !fits) & ((1ull << kWin) - 1);
    const int end = stop ? __builtin_ctzll(stop) : S.n0;
    const bool take = l >= i && l < end;  // consumed by this batch
    const int64_t q = S.base0 + l;
    if (take && a.status != nullptr) a.status[q] = LP.cls == CLS_NONE ? LP.st : 0;
    // quick returns (beta * C), one after another
    uint64_t qm = __ballot(take && LP.cls == CLS_QUICK);
    while (qm) {
      const int ql = __builtin_ctzll(qm);
      qm &= qm - 1;
      const Prob P = lane_prob_of(S.cur, ql);
      scale_columns(P.C, P.m, P.n, P.ldc, P.beta, 0, 1);
    }
    if (take && LP.cls == CLS_STAGE) {
      const int slot = np + c_cnt - 1;
      const int off = used + c_need - LP.need;  // staging offset of this problem
      const Prob P = lane_prob(S.cur);
      const int trans = (int)S.cur.w[6];
      const PcGeom g = pc_geom(P, trans & 1, trans >> 1);  // recomputed: fewer live registers
      BatchProb& bp = g_bprob[tb][slot];
      bp.C = P.C;
      bp.la = off + g.a_sh;
      bp.lb = off + 4 * g.a_n4 + g.b_sh;
      bp.lc = g.c_n4 > 0 ? off + 4 * (g.a_n4 + g.b_n4) + g.c_sh : -1;
      bp.m = P.m;
      bp.n = P.n;
      bp.k = P.k;
      bp.lda = P.lda;
      bp.ldb = P.ldb;
      bp.ldc = P.ldc;
      bp.alpha = P.alpha;
      bp.beta = P.beta;
      bp.trans = trans;
      CopyJob* cj = g_copy[tb] + 3 * slot;
      cj[0] = CopyJob{P.A - g.a_sh, off, g.a_n4};
      cj[1] = CopyJob{P.B - g.b_sh, off + 4 * g.a_n4, g.b_n4};
      cj[2] = CopyJob{P.C - g.c_sh, off + 4 * (g.a_n4 + g.b_n4), g.c_n4};
    }
    emit_units(S, LP, take, tb, np + c_cnt - 1, nlong + c_long - LP.nlong,
               kMaxUnits - 1 - ((nb - nlong) + (c_blk - c_long) - (LP.nbp - LP.nlong)));
    // totals of the taken lanes (lane end-1's prefix values; 0 if none)
    const int last = end - 1;
    if (last >= i) {
      used += __builtin_amdgcn_readlane(c_need, last);
      nb += __builtin_amdgcn_readlane(c_blk, last);
      nlong += __builtin_amdgcn_readlane(c_long, last);
      np += __builtin_amdgcn_readlane(c_cnt, last);
    }
    S.i = end;
    if (end < S.n0) break;  // a problem did not fit: this batch is full
  }
  if (l == 0) {
    g_bhead[tb][0] = np;
    g_bhead[tb][1] = nb;
    g_bhead[tb][2] = nlong;
    g_bhead[tb][3] = more ? 1 : 0;
  }
}

// Work-group barrier once this wavefront's staging copies have landed.
__device__ __forceinline__ void staged_barrier() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}

// Compute wavefront w (1..7) runs units w - 1, w + 6, w + 13, ... of the
// batch's longest-first unit list (a static round-robin: no claim round
// trip), reading the next unit word while the current unit runs.
__device__ __forceinline__ void compute_batch(int t, lds_f* stage, int nb, int nlong, int w) {
  const int gap = kMaxUnits - nb;  // unit b >= nlong sits at b + gap
  // static round-robin over the longest-first list: unit b to compute
  // wavefront (b mod 7); the next unit word is read while a unit runs
  int b = w - 1;
  uint32_t e_next = b < nb ? g_bunit[t][b < nlong ? b : b + gap] : 0u;
  while (b < nb) {
    const uint32_t e = rfl(e_next);
    const int bn = b + (kWaves - 1);
    e_next = bn < nb ? g_bunit[t][bn < nlong ? bn : bn + gap] : 0u;
    const int u = (int)((e >> 16) & 0xff), i0 = (int)(e & 0xff), j0 = (int)((e >> 8) & 0xff);
    const u4* pe = reinterpret_cast<const u4*>(&g_bprob[t][e >> 24]);
    const u4 w0 = pe[0], w1 = pe[1], w2 = pe[2], w3 = pe[3];
    float* C = (float*)(((uint64_t)rfl(w0.y) << 32) | rfl(w0.x));
    const int la = (int)rfl(w0.z), lb = (int)rfl(w0.w), lc = (int)rfl(w1.x);
    const int m = (int)rfl(w1.y), n = (int)rfl(w1.z), k = (int)rfl(w1.w);
    const int lda = (int)rfl(w2.x), ldb = (int)rfl(w2.y), ldc = (int)rfl(w2.z);
    const float alpha = __builtin_bit_cast(float, rfl(w2.w)), beta = __builtin_bit_cast(float, rfl(w3.x));
    const int trans = (int)rfl(w3.y);
    const SProb P{stage + la, stage + lb, lc >= 0 ? stage + lc : nullptr, C, m, n, k, lda, ldb, ldc,
                  ldc, alpha, beta};
    switch (trans) {
      case 0: run_unit<0, 0>(u, P, i0, j0); break;
      case 1: run_unit<1, 0>(u, P, i0, j0); break;
      case 2: run_unit<0, 1>(u, P, i0, j0); break;
      default: run_unit<1, 1>(u, P, i0, j0); break;
    }
    b = bn;
  }
}

// Every wavefront issues its share of batch t's copies: job c is cut into
// 64-unit chunks (one memory-to-LDS load instruction each); chunks are
// numbered across jobs and chunk q goes to wavefront q mod 8.  Lane c holds
// job c's entry (one LDS read).
__device__ __forceinline__ void issue_copies(int t, int w, lds_f* stage) {
  const int nc = 3 * uni(g_bhead[t][0]);  // three copy jobs per problem
  CopyJob my{};
  if (lane() < nc) my = g_copy[t][lane()];
  const uint64_t src_v = (uint64_t)my.src;
  int qbase = 0;
  for (int c = 0; c < nc; ++c) {
    const int n4 = rdl(my.n4, c);
    const int nch = (n4 + 63) >> 6;
    if (n4 > 0) {
      const uint64_t su = ((uint64_t)rdl((uint32_t)(src_v >> 32), c) << 32) | rdl((uint32_t)src_v, c);
      const float* g16 = (const float*)su;
      lds_f* dst = stage + rdl(my.dst, c);
      for (int ch = (w - qbase) & (kWaves - 1); ch < nch; ch += kWaves) {
        const int u = 64 * ch + lane();
        if (u < n4) copy16_lds(g16 + 4 * u, dst + 256 * ch);
      }
    }
    qbase += nch;
  }
}

// Iteration t: every wavefront issues its share of batch t's copies; one
// wait; wavefronts 1..7 compute batch t from LDS while wavefront 0 packs
// batch t+1 into the other table set (its own copies have landed, so its
// descriptor reads never wait behind them); a barrier closes the iteration
// because the staging buffer is refilled.  Wavefront 0 and the others run
// loops of their own with the same barriers, so the packer's state is not
// live in the compute code.
__device__ __forceinline__ void packer_loop(const VbArgs& a, lds_f* stage) {
  const WinShape z = win_shape(a);
  Windows S;
  S.end = false;
  S.t_last = 0;
  S.tk = 0;
  S.s1 = (int)z.s0;
  // this work-group's first window, fetched at once
  S.sbase = (int64_t)blockIdx.x * z.s0;
  S.base1 = S.sbase;
  S.n1 = (int)min<int64_t>(z.s0, z.count - S.sbase);
  window_load(S.nxt, a, S.base1, S.n1);
  window_load_plan(S.nxt, a.table);
  S.hop = 3;
  win_advance(S, a, z);
  pack_batch(a, z, S, 0);
  __syncthreads();  // batch 0's tables
  for (int t = 0;; t ^= 1) {
    const int more = uni(g_bhead[t][3]);
    issue_copies(t, 0, stage);
    staged_barrier();  // batch t has landed
    if (more) pack_batch(a, z, S, t ^ 1);
    if (!more) break;
    __syncthreads();  // batch t computed (buffer free); batch t+1's tables visible
  }
}

__device__ __forceinline__ void compute_loop(int w, lds_f* stage) {
  __syncthreads();  // batch 0's tables
  for (int t = 0;; t ^= 1) {
    const int np = uni(g_bhead[t][0]);
    const int nb = uni(g_bhead[t][1]);
    const int more = uni(g_bhead[t][3]);
    const int nlong = uni(g_bhead[t][2]);
    issue_copies(t, w, stage);
    staged_barrier();  // batch t has landed
    if (np > 0) compute_batch(t, stage, nb, nlong, w);
    if (!more) break;
    __syncthreads();
  }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
void vbatched_f32_kernel(VbArgs a) {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
  if ((int64_t)blockIdx.x * win_shape(a).s0 >= a.count) return;
  lds_f* stage = (lds_f*)g_stage;
  if (w == 0) packer_loop(a, stage);
  else compute_loop(w, stage);
}

__device__ __forceinline__ bool load_problem(const VbArgs& a, int64_t q, Prob& P, int& trans,
                                             int& st) {
  const iaat_problem* d = a.probs + q;
  trans = d->trans;
  P.m = d->m;
  P.n = d->n;
  P.k = d->k;
  P.lda = d->lda;
  P.ldb = d->ldb;
  P.ldc = d->ldc;
  P.alpha = d->alpha * d->ab_scale;
  P.beta = d->beta;
  P.A = (const float*)d->A;
  P.B = (const float*)d->B;
  P.C = d->C;
  st = validate(trans, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.A, P.B, P.C);
  return st == 0 && P.m > 0 && P.n > 0;
}

// Batched problems that do not fit the staging buffer.  Wavefront w of the
// grid screens problems 64w .. 64w + 63, one per lane (valid, needs A*B, and
// fails the same staging test as vbatched_f32_kernel, so every problem is
// computed by exactly one of the two kernels), then computes the ones found,
// one after another; most wavefronts find none and exit after one load.
__global__ __launch_bounds__(64) void vbatched_direct_kernel(VbArgs a) {
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int64_t q = base + lane();
  bool need = false;
  if (q < a.count) {
    Prob P;
    int trans, st;
    if (load_problem(a, q, P, trans, st) && P.alpha != 0.0f && P.k != 0)
      need = !pc_geom(P, trans & 1, trans >> 1).fits;
  }
  uint64_t mask = __ballot(need);
  while (mask) {
    const int l = __builtin_ctzll(mask);
    mask &= mask - 1;
    Prob P;
    int trans, st;
    load_problem(a, base + l, P, trans, st);
    direct_problem(trans, P, a.table);
  }
}


}  // namespace dev

hipError_t launch_vbatched_f32_staged(const VbArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::vbatched_f32_kernel, dim3((unsigned)grid), dim3(512), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int dgrid = (int)((a.count + 63) / 64);  // one screening wavefront per 64 problems
  hipLaunchKernelGGL(dev::vbatched_direct_kernel, dim3((unsigned)dgrid), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t vbatched_staged_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, dev::vbatched_f32_kernel, 512, 0);
}

}  // namespace iaat
