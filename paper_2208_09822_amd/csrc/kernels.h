// Host-side view of the device entry points (launch wrappers) of libiaat.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iaat_internal.h"

namespace iaat {
namespace dev {
// One FP32 problem (or super-block of one) as the block kernels see it;
// alpha already includes any dequantisation factor.
struct Prob {
  const float* A;
  const float* B;
  float* C;
  int m, n, k;
  int lda, ldb, ldc;  // each < 2^31
  float alpha, beta;
};
}  // namespace dev


struct VbArgs {
  const iaat_problem* probs;
  int64_t count;
  int32_t* status;
  const PlanEntry* table;
  uint32_t* ticket;  // NULL: windows dealt statically; else a counter handing them out
};

hipError_t launch_gemm_f32(const dev::Prob& P, int layout, const PlanEntry* table_dev, int nsm,
                           int nsn, int max_blocks, hipStream_t stream);
hipError_t launch_scale_f32(float* C, int m, int n, int ldc, float beta, hipStream_t stream);
hipError_t launch_gemm_f32_strided(const dev::Prob& P, int layout, const PlanEntry* table_dev, int nsm,
                                   int nsn, int max_blocks, int64_t sa, int64_t sb, int64_t sc,
                                   int64_t batch, hipStream_t stream);
// Descriptors (one iaat_problem per problem) of a same-size strided batch.
hipError_t launch_strided_desc(iaat_problem* d, int64_t batch, const dev::Prob& P, int layout,
                               int64_t sa, int64_t sb, int64_t sc, hipStream_t stream);
hipError_t launch_scale_f32_strided(float* C, int m, int n, int ldc, float beta, int64_t sc,
                                    int64_t batch, hipStream_t stream);
// The batched FP32 launch: a kernel clearing the ticket counter (when there
// is one), then the persistent batched kernel (batched.hip) on `grid`
// work-groups of 512 threads (two per CU) and its companion for problems too
// large to stage.
hipError_t launch_vbatched_f32(const VbArgs& a, int grid, hipStream_t stream);
hipError_t launch_vbatched_f32_staged(const VbArgs& a, int grid, hipStream_t stream);
hipError_t vbatched_occupancy(int* blocks_per_cu);
hipError_t vbatched_staged_occupancy(int* blocks_per_cu);

// Scratch of the allocation-free batched entry point (a file-scope device
// array in kernels.hip, kScratchWords 32-bit words).  scratch_init(device)
// takes its address on `device` (which must be current) once; afterwards
// scratch_address(device) returns it (NULL before scratch_init).
constexpr int kScratchWords = 64;
constexpr int kMaxDevices = 64;
hipError_t scratch_init(int device);
uint32_t* scratch_address(int device);


// Copies float spans (src, dst, n floats), one work-group per span.
struct CopySpan {
  const float* src;
  float* dst;
  int64_t n;
};
hipError_t launch_copy_spans(const CopySpan* spans, int64_t count, int grid, hipStream_t stream);

// DGEMM / CGEMM / ZGEMM (xgemm.hip): one problem or super-block as the
// family members see it; pointers to the stored matrices, dimensions in
// elements (complex elements for complex types), scalars in FP64 (rounded
// to FP32 for complex FP32).
struct XProb {
  const void* A;
  const void* B;
  void* C;
  int m, n, k, lda, ldb, ldc;
  double alpha_re, alpha_im, beta_re, beta_im;
};
// light: every block of the plans in use passes kid_is_light() (a kernel
// compiled with only those members, at a smaller register budget).
hipError_t launch_xgemm(int dt, const XProb& P, int layout, int64_t sa, int64_t sb, int64_t sc,
                        int64_t batch, const PlanEntry* table_dev, int nsm, int nsn, int max_blocks,
                        bool light, hipStream_t s);
hipError_t launch_xscale(int dt, const XProb& P, int64_t sc, int64_t batch, hipStream_t s);
hipError_t launch_xgemm_vbatched(int dt, const iaat_xproblem* probs, int64_t count, int32_t* status,
                                 const PlanEntry* table_dev, hipStream_t s);

// Traditional pack + uniform-tile scheme (traditional.hip), for ablation.
struct TradProb {
  const float* A;
  const float* B;
  float* C;
  int64_t a_off, b_off;  // packed op(A) / op(B) in the workspace, in floats
  int m, n, k, lda, ldb, ldc, trans;
  int m16, n16, k16;     // sizes rounded up to 16 (k16 = 0 when A and B are not read)
  float alpha, beta;
};
hipError_t launch_trad_pack(const TradProb* probs, int64_t count, float* work, int grid,
                            hipStream_t stream);
hipError_t launch_trad_tiles(const TradProb* probs, const int32_t* tiles, int64_t ntiles,
                             const float* work, int grid, hipStream_t stream);

// Reduced-precision inputs (precision.hip).
hipError_t launch_quantize(int prec, const iaat_qjob* jobs, int64_t count, int grid, hipStream_t stream);
hipError_t launch_vbatched_lowp(const VbArgs& a, int prec, int grid, hipStream_t stream);

}  // namespace iaat
