// Internal definitions shared by the host runtime and the device kernels of
// libiaat: problem validation (the argument rules of iaat_gemm), the
// small-GEMM domain test, and the tile-plan table format.
#pragma once

#include <stdint.h>

#include "../../include/iaat.h"
#include "generated/family.inc"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define IAAT_HD __host__ __device__ __forceinline__
#else
#define IAAT_HD inline
#endif

namespace iaat {

enum Family : int { FAM_MFMA = 0, FAM_ROWS = 1, FAM_COLS = 2, FAM_KRED = 3 };

// Largest (sub)problem a table plan covers; larger M or N are split into
// super-blocks of at most this size, each with its own table plan.
constexpr int kSuper = 80;
constexpr int kMaxBlocks = 15;
constexpr int kLayouts = 4;

// One table entry: the kernel executing plan (Section V-B) for a
// (layout, m, n) with 1 <= m, n <= 80.  64 bytes.
struct PlanEntry {
  uint32_t nblk;
  uint32_t blk[kMaxBlocks];  // i0 | j0 << 8 | kid << 16
};
static_assert(sizeof(PlanEntry) == 64, "plan entry must be 64 bytes");

IAAT_HD uint32_t pack_block(int i0, int j0, int kid) {
  return (uint32_t)i0 | ((uint32_t)j0 << 8) | ((uint32_t)kid << 16);
}
// Family members with a small register footprint: for real FP64 at most two
// matrix-core tiles, four strip rows or columns, four K-split outputs; for
// complex types one tile, two strip rows or columns, two K-split outputs.
// A kernel that holds only these keeps many wavefronts per SIMD; the FP64
// and complex launches use it when every block of a plan is one of them.
IAAT_HD constexpr bool kid_light(int fam, int p1, int p2, bool cplx) {
  return cplx ? (fam == 0 ? p1 * p2 <= 1 : fam == 1 ? p1 <= 2 : fam == 2 ? p2 <= 2 : p1 * p2 <= 2)
              : (fam == 0 ? p1 * p2 <= 2 : fam == 1 ? p1 <= 4 : fam == 2 ? p2 <= 4 : p1 * p2 <= 4);
}
IAAT_HD bool kid_is_light(int kid, bool cplx) {
  switch (kid) {
#define IAAT_LIGHT_CASE(id, fam, p1, p2, br, bc) \
  case id:                                     \
    return kid_light(fam, p1, p2, cplx);
    IAAT_FOR_EACH_KID(IAAT_LIGHT_CASE)
#undef IAAT_LIGHT_CASE
    default:
      return false;
  }
}
IAAT_HD int blk_i0(uint32_t b) { return (int)(b & 0xffu); }
IAAT_HD int blk_j0(uint32_t b) { return (int)((b >> 8) & 0xffu); }
IAAT_HD int blk_kid(uint32_t b) { return (int)((b >> 16) & 0xffu); }

IAAT_HD int plan_index(int layout, int m, int n) {
  return (layout * kSuper + (m - 1)) * kSuper + (n - 1);
}
constexpr int kPlanCount = kLayouts * kSuper * kSuper;

// Small-GEMM domain (Section I): cbrt(MNK) <= 80, <= 32 for TN, in exact
// integers.  Layout bit 0 = A^T, bit 1 = B^T, so TN is layout 1.
IAAT_HD bool in_small_domain(int layout, int64_t m, int64_t n, int64_t k) {
  const int64_t lim = (layout == 1) ? 32768 : 512000;
  if (m <= 0 || n <= 0 || k <= 0) return true;
  if (m > lim || n > lim || k > lim) return false;
  const int64_t mn = m * n;  // < 2^38
  if (mn > lim) return false;
  return mn * k <= lim;      // < 2^57
}

// Argument check of one problem; returns 0 or -(iaat_gemm argument number).
IAAT_HD int validate(int trans, int64_t m, int64_t n, int64_t k, int64_t lda, int64_t ldb,
                     int64_t ldc, float alpha, const void* A, const void* B, const void* C) {
  if (trans & ~3) return -3;
  const bool ta = trans & 1, tb = trans & 2;
  const int64_t lim = 0x7fffffffLL;
  if (m < 0 || m > lim) return -4;
  if (n < 0 || n > lim) return -5;
  if (k < 0 || k > lim) return -6;
  const int64_t ra = ta ? k : m, rb = tb ? n : k;
  if (lda < (ra > 1 ? ra : 1) || lda > lim) return -9;
  if (ldb < (rb > 1 ? rb : 1) || ldb > lim) return -11;
  if (ldc < (m > 1 ? m : 1) || ldc > lim) return -14;
  if (m == 0 || n == 0) return 0;
  const bool reads_ab = (alpha != 0.0f) && (k > 0);
  if (reads_ab && A == nullptr) return -8;
  if (reads_ab && B == nullptr) return -10;
  if (C == nullptr) return -13;
  return 0;
}

}  // namespace iaat
