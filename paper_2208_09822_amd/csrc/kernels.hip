// Device entry points of libiaat: the per-call kernel (one problem, one
// work-group per block of its tile plan), the persistent batched kernel
// (wavefronts pop whole problems from a device work queue and run each
// problem's kernel executing plan), and the quick-return scaling kernel.
#include <hip/hip_runtime.h>

#include "iaat_internal.h"
#include "kernels.h"
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

__global__ void zero_u32_kernel(uint32_t* p, int n) {
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = 0u;
}

__device__ __forceinline__ void batched_problem(const VbArgs& a, int64_t q) {
  const iaat_problem* d = a.probs + q;
  const int trans = d->trans;
  const int m = d->m, n = d->n, k = d->k;
  const int lda = d->lda, ldb = d->ldb, ldc = d->ldc;
  const float alpha = d->alpha * d->ab_scale, beta = d->beta;
  const float* A = (const float*)d->A;
  const float* B = (const float*)d->B;
  float* C = d->C;
  const int st = validate(trans, m, n, k, lda, ldb, ldc, alpha, A, B, C);
  if (a.status != nullptr && lane() == 0) a.status[q] = st;
  if (st != 0 || m == 0 || n == 0) return;
  if (alpha == 0.0f || k == 0) {
    scale_columns(C, m, n, ldc, beta, 0, 1);
    return;
  }
  const Prob P{A, B, C, m, n, k, lda, ldb, ldc, alpha, beta};
  switch (trans) {
    case 0: solve_problem<0, 0>(P, a.table); break;
    case 1: solve_problem<1, 0>(P, a.table); break;
    case 2: solve_problem<0, 1>(P, a.table); break;
    default: solve_problem<1, 1>(P, a.table); break;
  }
}

// Persistent batched kernel.  The problem list is cut into 8 contiguous
// ranges with one queue counter each (work-group w starts on range w % 8,
// the XCD it is dispatched to); a wavefront pops problems from its range
// until it is empty and then helps the other ranges in turn, so every
// wavefront exits once all counters have passed their range ends.  The last
// wavefront to finish (counted on a ninth counter) sets all counters back to
// zero for the next launch that uses this counter slot.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4))) void vbatched_f32_kernel(VbArgs a) {
  const int home = (int)(blockIdx.x & 7);
  for (int rr = 0; rr < 8; ++rr) {
    const int x = (home + rr) & 7;
    const int64_t lo = a.count * x / 8, hi = a.count * (x + 1) / 8;
    if (lo >= hi) continue;
    for (;;) {
      uint32_t t = 0;
      if (lane() == 0) t = atomicAdd(a.ctr + x * kCtrStride, 1u);
      t = __builtin_amdgcn_readfirstlane(t);
      const int64_t q = lo + (int64_t)t;
      if (q >= hi) break;
      batched_problem(a, q);
    }
  }
  if (lane() == 0) {
    // acq_rel: this wavefront's last pop (whose result it has already used)
    // is ordered before its count, and the resets after all counts
    const uint32_t done = __hip_atomic_fetch_add(a.ctr + 8 * kCtrStride, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {  // every other wavefront has left its loop
      for (int x = 0; x <= 8; ++x)
        __hip_atomic_exchange(a.ctr + x * kCtrStride, 0u, __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace dev

// ------------------------------------------------------------ host launchers

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

hipError_t launch_scale_f32(float* C, int m, int n, int ldc, float beta, hipStream_t stream) {
  const unsigned g = (unsigned)(n < 65536 ? n : 65536);
  hipLaunchKernelGGL(dev::scale_kernel, dim3(g), dim3(64), 0, stream, C, m, n, ldc, beta);
  return hipGetLastError();
}

hipError_t launch_zero_u32(uint32_t* p, int n, hipStream_t stream) {
  hipLaunchKernelGGL(dev::zero_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_vbatched_f32(const VbArgs& a, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::vbatched_f32_kernel, dim3((unsigned)grid), dim3(64), 0, stream, a);
  return hipGetLastError();
}

hipError_t vbatched_occupancy(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, dev::vbatched_f32_kernel, 64, 0);
}

}  // namespace iaat
