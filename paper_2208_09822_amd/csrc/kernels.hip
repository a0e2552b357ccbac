// Device entry points of libiaat: the per-call kernel (one problem, one
// work-group per block of its tile plan), its same-size strided form, the
// batched kernels (work-groups stage batches of problems in LDS and run
// their kernel executing plans from there; problems too large to stage go
// to a direct kernel), the quick-return scaling kernels and the span copy
// used by the serving loop.
#include <hip/hip_runtime.h>

#include <mutex>

#include "iaat_internal.h"
#include "kernels.h"
#include "lds_tiles.h"
#include "tiles.h"

namespace iaat {
namespace dev {

// Dispatch one block to its generated kernel.  The switch is uniform per
// wavefront (kid comes from the plan table), so it never diverges.
template <int TA, int TB>
__device__ __forceinline__ void run_block(int kid, const Prob& P, int i0, int j0) {
  switch (kid) {
#define IAAT_CASE(id, fam, p1, p2, br, bc) \
  case id:                                  \
    BlockOp<fam, TA, TB, p1, p2>::run(P, i0, j0); \
    break;
    IAAT_FOR_EACH_KID(IAAT_CASE)
#undef IAAT_CASE
    default:
      break;
  }
}

// The part of a problem covered by super-block (sbi, sbj): rows
// [80 sbi, 80 sbi + 80) and columns [80 sbj, 80 sbj + 80) of C.  K is never
// split, so A keeps all of its K extent (Section V-A).
template <int TA, int TB>
__device__ __forceinline__ Prob sub_problem(const Prob& P, int sbi, int sbj) {
  Prob S = P;
  const int64_t r0 = (int64_t)sbi * kSuper, c0 = (int64_t)sbj * kSuper;
  S.A = TA ? P.A + r0 * P.lda : P.A + r0;
  S.B = TB ? P.B + c0 : P.B + c0 * P.ldb;
  S.C = P.C + r0 + c0 * P.ldc;
  S.m = (int)min((int64_t)kSuper, (int64_t)P.m - r0);
  S.n = (int)min((int64_t)kSuper, (int64_t)P.n - c0);
  return S;
}

__device__ __forceinline__ bool narrow(const Prob& P) {
  return P.lda <= kNarrowLd && P.ldb <= kNarrowLd && P.ldc <= kNarrowLd;
}

// Whole problem on one wavefront: every super-block, every block of its plan.
template <int TA, int TB>
__device__ __forceinline__ void solve_problem(const Prob& P, const PlanEntry* __restrict__ table) {
  const int layout = TA | (TB << 1);
  const int nsm = (P.m + kSuper - 1) / kSuper, nsn = (P.n + kSuper - 1) / kSuper;
  const bool nar = narrow(P);
  for (int sbj = 0; sbj < nsn; ++sbj)
    for (int sbi = 0; sbi < nsm; ++sbi) {
      const Prob S = sub_problem<TA, TB>(P, sbi, sbj);
      if (!nar) {
        wide_subproblem<TA, TB>(S);
        continue;
      }
      const PlanEntry* e = table + plan_index(layout, S.m, S.n);
      const int nb = (int)e->nblk;
      for (int b = 0; b < nb; ++b) {
        const uint32_t w = e->blk[b];
        run_block<TA, TB>(blk_kid(w), S, blk_i0(w), blk_j0(w));
      }
    }
}

// One problem per call: grid.x = super-blocks, grid.y = block slot in plan.
template <int TA, int TB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f32_kernel(Prob P, const PlanEntry* __restrict__ table,
                                                      int nsn) {
  const int sb = blockIdx.x, b = blockIdx.y;
  const int sbi = sb / nsn, sbj = sb - sbi * nsn;
  const Prob S = sub_problem<TA, TB>(P, sbi, sbj);
  if (!narrow(P)) {
    if (b == 0) wide_subproblem<TA, TB>(S);
    return;
  }
  const PlanEntry* e = table + plan_index(TA | (TB << 1), S.m, S.n);
  if (b >= (int)e->nblk) return;
  const uint32_t w = e->blk[b];
  run_block<TA, TB>(blk_kid(w), S, blk_i0(w), blk_j0(w));
}

// C = beta*C (alpha == 0 or K == 0); each work-group takes columns.
__global__ __launch_bounds__(64) void scale_kernel(float* C, int m, int n, int ldc, float beta) {
  scale_columns(C, m, n, ldc, beta, (int)blockIdx.x, (int)gridDim.x);
}

// Same-size batch: problem z has operands at A + z*sa, B + z*sb, C + z*sc;
// grid.z walks the problems (grid-stride), grid.x/y as in gemm_f32_kernel,
// with the one plan every problem shares.
template <int TA, int TB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_f32_strided_kernel(
    Prob P, int64_t sa, int64_t sb, int64_t sc, int64_t batch, const PlanEntry* __restrict__ table,
    int nsn) {
  const int sbk = blockIdx.x, b = blockIdx.y;
  const int sbi = sbk / nsn, sbj = sbk - sbi * nsn;
  const bool nar = narrow(P);
  const PlanEntry* e = table + plan_index(TA | (TB << 1), sub_problem<TA, TB>(P, sbi, sbj).m,
                                          sub_problem<TA, TB>(P, sbi, sbj).n);
  if (nar ? b >= (int)e->nblk : b > 0) return;
  for (int64_t z = blockIdx.z; z < batch; z += gridDim.z) {
    Prob Q = P;
    Q.A += z * sa;
    Q.B += z * sb;
    Q.C += z * sc;
    const Prob S = sub_problem<TA, TB>(Q, sbi, sbj);
    if (!nar) {
      wide_subproblem<TA, TB>(S);
      continue;
    }
    const uint32_t w = e->blk[b];
    run_block<TA, TB>(blk_kid(w), S, blk_i0(w), blk_j0(w));
  }
}

__global__ __launch_bounds__(64) void scale_strided_kernel(float* C, int m, int n, int ldc, float beta,
                                                           int64_t sc, int64_t batch) {
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y)
    scale_columns(C + z * sc, m, n, ldc, beta, (int)blockIdx.x, (int)gridDim.x);
}

// ---------------------------------------------------------------------------
// Batched path.

// Kernel family parameters, indexed by kid.
__constant__ int kKidFam[IAAT_NUM_KIDS] = {
#define IAAT_F(id, fam, p1, p2, br, bc) fam,
    IAAT_FOR_EACH_KID(IAAT_F)
#undef IAAT_F
};
__constant__ int kKidP1[IAAT_NUM_KIDS] = {
#define IAAT_F(id, fam, p1, p2, br, bc) p1,
    IAAT_FOR_EACH_KID(IAAT_F)
#undef IAAT_F
};
__constant__ int kKidP2[IAAT_NUM_KIDS] = {
#define IAAT_F(id, fam, p1, p2, br, bc) p2,
    IAAT_FOR_EACH_KID(IAAT_F)
#undef IAAT_F
};

// ---- batched kernel: staged batches --------------------------------------
//
// Work-groups of eight wavefronts, two per CU (each owns half of the LDS).
// Problems go to work-groups in windows of kWin consecutive problems: window
// w to work-group w mod G, or, with a ticket counter, the first G windows so
// and the rest to whichever work-group asks next (balancing the uneven
// work).  Wavefront 0 packs a batch -- as many of the work-group's next
// problems as fit into its staging buffer, one problem per lane, the
// descriptors read a window ahead -- into one of two table sets.  Every
// wavefront copies its share of the batch's A, B and (when beta != 0) C
// spans verbatim into LDS with memory-to-LDS loads; after one wait,
// wavefronts 1..7 run the batch's plan blocks round-robin from LDS and store
// C while wavefront 0 packs the next batch.  A barrier closes the iteration
// because the buffer is refilled.  Problems that do not fit the buffer are
// left to vbatched_direct_kernel; quick returns and status codes are handled
// here.

constexpr int kStage = 19440;        // floats of staging per work-group (>= one 80x80x80 problem)
constexpr int kMaxBatch = 16;        // problems per batch
constexpr int kMaxBatchBlocks = 64;  // plan blocks per batch
constexpr int kWaves = 8;
constexpr int kWin = 4;              // problems per descriptor window

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
__shared__ BatchProb g_bprob[2][kMaxBatch];
__shared__ uint32_t g_bblk[2][kMaxBatchBlocks];  // plan block | problem slot << 24
__shared__ CopyJob g_copy[2][3 * kMaxBatch];
__shared__ int g_bhead[2][4];                    // problems, blocks, copies, more-to-come

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

// Staged-operand dispatch: one routine per scheme, the kernel's sizes passed
// as run-time values (each stored element gets the same arithmetic as in the
// specialised direct kernels).
template <int TA, int TB>
__device__ __forceinline__ void run_block_lds(int kid, const LdsProb& P, int i0, int j0, int sync) {
  const int fam = kKidFam[kid], p1 = kKidP1[kid], p2 = kKidP2[kid];
  if (fam == FAM_MFMA) LdsMfma<TA, TB>::run(P, i0, j0, sync, p1, p2);
  else if (fam == FAM_ROWS) LdsRows<TA, TB>::run(P, i0, j0, sync, p1);
  else if (fam == FAM_COLS) LdsCols<TA, TB>::run(P, i0, j0, sync, p2);
  else LdsKred<TA, TB>::run(P, i0, j0, sync, p1, p2);
}

// One 16-byte memory-to-LDS load: this lane's 16 bytes land at `base` + 16 *
// lane (`base` is the same for the whole wavefront).
__device__ __forceinline__ void copy16_lds(const float* g16, lds_f* base) {
  typedef __attribute__((address_space(1))) const void gvoid;
  typedef __attribute__((address_space(3))) void lvoid;
  __builtin_amdgcn_global_load_lds((gvoid*)g16, (lvoid*)base, 16, 0, 0);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ const void* unip(const void* p) {
  const uint64_t v = (uint64_t)p;
  return (const void*)(((uint64_t)(uint32_t)uni((int)(v >> 32)) << 32) | (uint32_t)uni((int)v));
}

__device__ __forceinline__ int rdl(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint32_t rdl(uint32_t v, int l) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ float rdlf(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// kWin descriptors (lane l < kWin holds problem base + l) and plan heads.
struct DescWindow {
  uint32_t w[16];  // the iaat_problem words
  uint32_t nblk, b0, b1, b2, b3;
};

__device__ __forceinline__ void window_load(DescWindow& W, const VbArgs& a, int64_t base) {
  const int64_t q = min(base + (lane() & (kWin - 1)), a.count - 1);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(a.probs + q);
#pragma unroll
  for (int i = 0; i < 16; ++i) W.w[i] = src[i];
}

__device__ __forceinline__ void window_load_plan(DescWindow& W, const PlanEntry* table) {
  const int trans = (int)W.w[6];
  const int m = min(max((int)W.w[7], 1), kSuper), n = min(max((int)W.w[8], 1), kSuper);
  const PlanEntry* e = table + plan_index(trans & 3, m, n);
  W.nblk = e->nblk;
  W.b0 = e->blk[0];
  W.b1 = e->blk[1];
  W.b2 = e->blk[2];
  W.b3 = e->blk[3];
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
  int cls, st, need, nbp;
  PcGeom g;
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
    r.g = pc_geom(P, trans & 1, trans >> 1);
    r.cls = r.g.fits ? CLS_STAGE : CLS_DIRECT;
    r.need = r.g.fits ? 4 * (r.g.a_n4 + r.g.b_n4 + r.g.c_n4) : 0;
    r.nbp = r.g.fits ? (int)W.nblk : 0;
  }
  return r;
}

// Inclusive prefix sum over the first kWin lanes.
__device__ __forceinline__ int scan16(int v) {
  const int l = lane();
#pragma unroll
  for (int off = 1; off < kWin; off <<= 1) {
    const int u = __shfl_up(v, off, 64);
    if (l >= off) v += u;
  }
  return v;
}

// The window after `win` for this work-group: the next of its static share
// (window w to work-group w mod G), or -- with a ticket counter -- the next
// window not yet handed out (windows 0..G-1 go to work-groups 0..G-1 first).
__device__ __forceinline__ int64_t next_window(const VbArgs& a, int64_t win, int64_t G) {
  if (a.ticket == nullptr) return win + G;
  uint32_t t = 0;
  if (lane() == 0) t = atomicAdd(a.ticket, 1u);
  return G + (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)t);
}

// Wavefront 0 packs the next batch: problems of this work-group's windows,
// in order, while they fit.  All bookkeeping is per lane (one problem per
// lane) plus prefix sums, then every taken lane writes its own table
// entries; so the cost per batch does not grow with the number of problems.
__device__ __forceinline__ void pack_batch(const VbArgs& a, int64_t G, int64_t nwin, int64_t& win,
                                           int64_t& win1, int& i, DescWindow& W0, DescWindow& W1,
                                           LaneProb& LP, int tb) {
  const int l = lane();
  int used = 0, np = 0, nb = 0, nc = 0;
  bool more = true;
  for (;;) {
    if (i == kWin) {  // window done: W1 holds window win1's words, read one window ahead
      win = win1;
      if (win >= nwin) {
        more = false;
        break;
      }
      window_load_plan(W1, a.table);
      W0 = W1;
      i = 0;
      LP = classify(W0, l < kWin && win * kWin + l < a.count);
      win1 = next_window(a, win, G);
      if (win1 < nwin) window_load(W1, a, win1 * kWin);
    }
    // candidates: lanes >= i that are staged
    const bool cand = l >= i && l < kWin && LP.cls == CLS_STAGE;
    const int c_need = scan16(cand ? LP.need : 0);
    const int c_blk = scan16(cand ? LP.nbp : 0);
    const int c_cnt = scan16(cand ? 1 : 0);
    const bool fits = used + c_need <= kStage && nb + c_blk <= kMaxBatchBlocks && np + c_cnt <= kMaxBatch;
    // first staged lane that does not fit ends this batch
    const uint64_t stop = __ballot(cand && !fits) & ((1ull << kWin) - 1);
    const int end = stop ? __builtin_ctzll(stop) : kWin;
    const bool take = l >= i && l < end;  // consumed by this batch
    const int64_t q = win * kWin + l;
    if (take && LP.cls != CLS_NONE && a.status != nullptr) a.status[q] = 0;
    if (take && LP.cls == CLS_NONE && l < kWin && q < a.count && a.status != nullptr) a.status[q] = LP.st;
    // quick returns (beta * C), one after another
    uint64_t qm = __ballot(take && LP.cls == CLS_QUICK);
    while (qm) {
      const int ql = __builtin_ctzll(qm);
      qm &= qm - 1;
      const Prob P = lane_prob_of(W0, ql);
      scale_columns(P.C, P.m, P.n, P.ldc, P.beta, 0, 1);
    }
    if (take && LP.cls == CLS_STAGE) {
      const int slot = np + c_cnt - 1;
      const int off = used + c_need - LP.need;  // staging offset of this problem
      const Prob P = lane_prob(W0);
      const PcGeom& g = LP.g;
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
      bp.trans = (int)W0.w[6];
      CopyJob* cj = g_copy[tb] + 3 * slot;
      cj[0] = CopyJob{P.A - g.a_sh, off, g.a_n4};
      cj[1] = CopyJob{P.B - g.b_sh, off + 4 * g.a_n4, g.b_n4};
      cj[2] = CopyJob{P.C - g.c_sh, off + 4 * (g.a_n4 + g.b_n4), g.c_n4};
      const int b0 = nb + c_blk - LP.nbp;
      const uint32_t tag = (uint32_t)slot << 24;
      uint32_t* bb = g_bblk[tb] + b0;
      if (LP.nbp > 0) bb[0] = W0.b0 | tag;
      if (LP.nbp > 1) bb[1] = W0.b1 | tag;
      if (LP.nbp > 2) bb[2] = W0.b2 | tag;
      if (LP.nbp > 3) bb[3] = W0.b3 | tag;
      if (LP.nbp > 4) {
        const PlanEntry* e = a.table + plan_index((int)W0.w[6] & 3, P.m, P.n);
        for (int b = 4; b < LP.nbp; ++b) bb[b] = e->blk[b] | tag;
      }
    }
    // totals of the taken lanes (lane end-1's prefix values; 0 if none)
    const int last = end - 1;
    const int t_need = last >= i ? __builtin_amdgcn_readlane(c_need, last) : 0;
    const int t_blk = last >= i ? __builtin_amdgcn_readlane(c_blk, last) : 0;
    const int t_cnt = last >= i ? __builtin_amdgcn_readlane(c_cnt, last) : 0;
    used += t_need;
    nb += t_blk;
    np += t_cnt;
    nc = 3 * np;
    i = end;
    if (end < kWin) break;  // a problem did not fit: this batch is full
  }
  if (l == 0) {
    g_bhead[tb][0] = np;
    g_bhead[tb][1] = nb;
    g_bhead[tb][2] = nc;
    g_bhead[tb][3] = more ? 1 : 0;
  }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4, 4)))
void vbatched_f32_kernel(VbArgs a) {
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
  const int64_t G = gridDim.x;
  const int64_t nwin = (a.count + kWin - 1) / kWin;
  int64_t win = blockIdx.x;  // this work-group's current window (wavefront 0's state)
  if (win >= nwin) return;
  DescWindow W0, W1;
  LaneProb LP{};
  int i = 0;
  int64_t win1 = 0;  // the window after win (its words in W1)
  if (w == 0) {
    window_load(W0, a, win * kWin);
    window_load_plan(W0, a.table);
    win1 = next_window(a, win, G);
    if (win1 < nwin) window_load(W1, a, win1 * kWin);
    LP = classify(W0, lane() < kWin && win * kWin + lane() < a.count);
    pack_batch(a, G, nwin, win, win1, i, W0, W1, LP, 0);
  }
  lds_f* stage = (lds_f*)g_stage;
  __syncthreads();  // batch 0's tables
  // Iteration t: every wavefront issues its share of batch t's copies; one
  // wait; wavefronts 1..7 compute batch t from LDS while wavefront 0 packs
  // batch t+1 into the other table set (its own copies have landed, so its
  // descriptor reads never wait behind them); a barrier closes the
  // iteration because the staging buffer is refilled.
  for (int t = 0;; t ^= 1) {
    const int np = uni(g_bhead[t][0]);
    const int nb = uni(g_bhead[t][1]);
    const int nc = uni(g_bhead[t][2]);
    const int more = uni(g_bhead[t][3]);
    if (np > 0) {
      // Copies: job c is cut into 64-unit chunks (one memory-to-LDS load
      // instruction each); chunks are numbered across jobs and chunk q goes
      // to wavefront q mod 8.  Lane c holds job c's entry (one LDS read).
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
    staged_barrier();  // batch t has landed
    if (w == 0) {
      if (more) pack_batch(a, G, nwin, win, win1, i, W0, W1, LP, t ^ 1);
    } else if (np > 0) {
      // blocks c, c + 7, ... on compute wavefront c = w - 1: lane u holds block c + 7u
      constexpr int kCompute = kWaves - 1;
      const int c0 = w - 1;
      const int myb = c0 + kCompute * lane();
      const uint32_t e_v = myb < nb ? g_bblk[t][myb] : 0u;
      for (int u = 0; c0 + kCompute * u < nb; ++u) {
        const uint32_t e = rdl(e_v, u);
        const BatchProb& bp = g_bprob[t][e >> 24];
        const int lc = uni(bp.lc);
        const LdsProb L{stage + uni(bp.la), stage + uni(bp.lb), lc >= 0 ? stage + lc : nullptr,
                        (float*)unip(bp.C), uni(bp.m), uni(bp.n), uni(bp.k), uni(bp.lda),
                        uni(bp.ldb), uni(bp.ldc), unif(bp.alpha), unif(bp.beta)};
        const int trans = uni(bp.trans);
        const int kid = blk_kid(e), i0 = blk_i0(e), j0 = blk_j0(e);
        switch (trans) {
          case 0: run_block_lds<0, 0>(kid, L, i0, j0, SYNC_NONE); break;
          case 1: run_block_lds<1, 0>(kid, L, i0, j0, SYNC_NONE); break;
          case 2: run_block_lds<0, 1>(kid, L, i0, j0, SYNC_NONE); break;
          default: run_block_lds<1, 1>(kid, L, i0, j0, SYNC_NONE); break;
        }
      }
    }
    if (!more) break;
    __syncthreads();  // batch t computed (buffer free); batch t+1's tables visible
  }
}

// A problem that does not fit the staging buffer, on one wavefront: every
// super-block, every block of its plan, operands read straight from memory.
// A separate function per layout (this path is rare; keeping it out of line
// keeps the batched kernels small).  Arguments are wave-uniform and are made
// scalar again on entry.
template <int TA, int TB>
__device__ __noinline__ void direct_problem_fn(const float* A, const float* B, float* C, int m, int n,
                                               int k, int lda, int ldb, int ldc, float alpha,
                                               float beta, const PlanEntry* table) {
  const Prob P{(const float*)unip(A), (const float*)unip(B), (float*)unip(C), uni(m), uni(n), uni(k),
               uni(lda), uni(ldb), uni(ldc), unif(alpha), unif(beta)};
  solve_problem<TA, TB>(P, (const PlanEntry*)unip(table));
}

template <int TA, int TB>
__device__ __forceinline__ void direct_problem(const Prob& P, const PlanEntry* __restrict__ table) {
  direct_problem_fn<TA, TB>(P.A, P.B, P.C, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.beta, table);
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
    switch (trans) {
      case 0: direct_problem<0, 0>(P, a.table); break;
      case 1: direct_problem<1, 0>(P, a.table); break;
      case 2: direct_problem<0, 1>(P, a.table); break;
      default: direct_problem<1, 1>(P, a.table); break;
    }
  }
}

// Clears a ticket counter (a kernel, so a captured graph holds no memset node).
__global__ __launch_bounds__(64) void clear_ticket_kernel(uint32_t* t) {
  if (threadIdx.x == 0) *t = 0;
}

__global__ __launch_bounds__(256) void copy_spans_kernel(const CopySpan* spans, int64_t count) {
  for (int64_t j = blockIdx.x; j < count; j += gridDim.x) {
    const CopySpan S = spans[j];
    for (int64_t i = threadIdx.x; i < S.n; i += blockDim.x) S.dst[i] = S.src[i];
  }
}

// Device scratch of the allocation-free batched entry point: word 0 is the
// window counter that hands 4-problem windows out to work-groups.  Each GPU
// the library runs on holds its own copy until the process ends.  In host
// code the name is only a stand-in: the device address comes from
// scratch_address(), taken once per device.
static __device__ __align__(256) uint32_t scratch[kScratchWords];

}  // namespace dev

// ------------------------------------------------------------ host launchers

namespace {
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device] != nullptr) return hipSuccess;
  // the caller made `device` current
  uint32_t* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(dev::scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

uint32_t* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_copy_spans(const CopySpan* spans, int64_t count, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::copy_spans_kernel, dim3((unsigned)grid), dim3(256), 0, stream, spans, count);
  return hipGetLastError();
}

hipError_t launch_gemm_f32(const dev::Prob& P, int layout, const PlanEntry* table_dev, int nsm,
                           int nsn, int max_blocks, hipStream_t stream) {
  const dim3 grid((unsigned)(nsm * nsn), (unsigned)max_blocks), block(64);
  switch (layout) {
    case 0: hipLaunchKernelGGL((dev::gemm_f32_kernel<0, 0>), grid, block, 0, stream, P, table_dev, nsn); break;
    case 1: hipLaunchKernelGGL((dev::gemm_f32_kernel<1, 0>), grid, block, 0, stream, P, table_dev, nsn); break;
    case 2: hipLaunchKernelGGL((dev::gemm_f32_kernel<0, 1>), grid, block, 0, stream, P, table_dev, nsn); break;
    default: hipLaunchKernelGGL((dev::gemm_f32_kernel<1, 1>), grid, block, 0, stream, P, table_dev, nsn); break;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_f32_strided(const dev::Prob& P, int layout, const PlanEntry* table_dev, int nsm,
                                   int nsn, int max_blocks, int64_t sa, int64_t sb, int64_t sc,
                                   int64_t batch, hipStream_t stream) {
  const unsigned gz = (unsigned)(batch < 65535 ? batch : 65535);
  const dim3 grid((unsigned)(nsm * nsn), (unsigned)max_blocks, gz), block(64);
  switch (layout) {
    case 0: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<0, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, table_dev, nsn); break;
    case 1: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<1, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, table_dev, nsn); break;
    case 2: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<0, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, table_dev, nsn); break;
    default: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<1, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, table_dev, nsn); break;
  }
  return hipGetLastError();
}

hipError_t launch_scale_f32_strided(float* C, int m, int n, int ldc, float beta, int64_t sc,
                                    int64_t batch, hipStream_t stream) {
  const unsigned gx = (unsigned)(n < 64 ? n : 64), gy = (unsigned)(batch < 65535 ? batch : 65535);
  hipLaunchKernelGGL(dev::scale_strided_kernel, dim3(gx, gy), dim3(64), 0, stream, C, m, n, ldc, beta, sc, batch);
  return hipGetLastError();
}

hipError_t launch_scale_f32(float* C, int m, int n, int ldc, float beta, hipStream_t stream) {
  const unsigned g = (unsigned)(n < 65536 ? n : 65536);
  hipLaunchKernelGGL(dev::scale_kernel, dim3(g), dim3(64), 0, stream, C, m, n, ldc, beta);
  return hipGetLastError();
}

hipError_t launch_vbatched_f32(const VbArgs& a, int grid, int direct_grid, hipStream_t stream) {
  if (a.ticket != nullptr) {
    hipLaunchKernelGGL(dev::clear_ticket_kernel, dim3(1), dim3(64), 0, stream, a.ticket);
    const hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  hipLaunchKernelGGL(dev::vbatched_f32_kernel, dim3((unsigned)grid), dim3(512), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dev::vbatched_direct_kernel, dim3((unsigned)direct_grid), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t vbatched_occupancy(int* blocks_per_cu, int* direct_per_cu) {
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, dev::vbatched_f32_kernel, 512, 0);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(direct_per_cu, dev::vbatched_direct_kernel, 64, 0);
}

}  // namespace iaat
