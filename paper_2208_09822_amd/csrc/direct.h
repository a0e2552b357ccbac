// Direct-from-memory execution of whole problems: super-block splitting,
// plan lookup and dispatch of each plan block to its generated kernel
// (tiles.h).  Used by the per-call and strided kernels (one block per
// work-group) and by the batched kernel for problems it does not stage.
#pragma once

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

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ const void* unip(const void* p) {
  const uint64_t v = (uint64_t)p;
  return (const void*)(((uint64_t)(uint32_t)uni((int)(v >> 32)) << 32) | (uint32_t)uni((int)v));
}

// A problem computed straight from memory on one wavefront (every
// super-block, every block of its plan).  A separate function per layout,
// kept out of line: this path is rare, and inlining it would bloat the
// kernels that call it.  Arguments are wave-uniform and are made scalar
// again on entry.
template <int TA, int TB>
__device__ __noinline__ void direct_problem_fn(const float* A, const float* B, float* C, int m, int n,
                                               int k, int lda, int ldb, int ldc, float alpha,
                                               float beta, const PlanEntry* table) {
  const Prob P{(const float*)unip(A), (const float*)unip(B), (float*)unip(C), uni(m), uni(n), uni(k),
               uni(lda), uni(ldb), uni(ldc), unif(alpha), unif(beta)};
  solve_problem<TA, TB>(P, (const PlanEntry*)unip(table));
}

__device__ __forceinline__ void direct_problem(int trans, const Prob& P, const PlanEntry* table) {
  switch (trans) {
    case 0: direct_problem_fn<0, 0>(P.A, P.B, P.C, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.beta, table); break;
    case 1: direct_problem_fn<1, 0>(P.A, P.B, P.C, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.beta, table); break;
    case 2: direct_problem_fn<0, 1>(P.A, P.B, P.C, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.beta, table); break;
    default: direct_problem_fn<1, 1>(P.A, P.B, P.C, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.beta, table); break;
  }
}

}  // namespace dev
}  // namespace iaat
