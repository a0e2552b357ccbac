// Device entry points of libiaat: the per-call kernel (one problem, one
// work-group per block of its tile plan), its same-size strided form, the
// quick-return scaling kernels, the ticket clear that precedes each batched
// launch (the batched kernel itself is in batched.hip) and the span copy
// used by the serving loop.
#include <hip/hip_runtime.h>

#include <mutex>

#include "iaat_internal.h"
#include "kernels.h"
#include "direct.h"
#include "tiles.h"

namespace iaat {
namespace dev {

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

// Same-size batch: problem z has operands at A + z*sa, B + z*sb, C + z*sc,
// with the one plan every problem shares.  One plan block of one
// super-block of one problem per work-group: grid.x = problem * slots +
// block slot (a problem's blocks side by side), grid.y = super-block - sb0;
// the host launches very long batches in pieces.  There is no loop over the
// batch: a loop around the block switch raises the registers it takes.
template <int TA, int TB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void gemm_f32_strided_kernel(
    Prob P, int64_t sa, int64_t sb, int64_t sc, int64_t batch, const PlanEntry* __restrict__ table,
    int nsn, int sb0, int slots) {
  const int sbk = sb0 + (int)blockIdx.y, b = (int)(blockIdx.x % (unsigned)slots);
  const int64_t z = blockIdx.x / (unsigned)slots;
  if (z >= batch) return;
  const int sbi = sbk / nsn, sbj = sbk - sbi * nsn;
  const bool nar = narrow(P);
  const PlanEntry* e = table + plan_index(TA | (TB << 1), sub_problem<TA, TB>(P, sbi, sbj).m,
                                          sub_problem<TA, TB>(P, sbi, sbj).n);
  if (nar ? b >= (int)e->nblk : b > 0) return;
  Prob Q = P;
  Q.A += z * sa;
  Q.B += z * sb;
  Q.C += z * sc;
  const Prob S = sub_problem<TA, TB>(Q, sbi, sbj);
  if (!nar) {
    wide_subproblem<TA, TB>(S);
    return;
  }
  const uint32_t w = e->blk[b];
  run_block<TA, TB>(blk_kid(w), S, blk_i0(w), blk_j0(w));
}

// Descriptors of a same-size strided batch (problem z at A + z*sa, ...), for
// the staged batched kernel.
__global__ __launch_bounds__(256) void strided_desc_kernel(iaat_problem* d, int64_t batch, Prob P,
                                                           int trans, int64_t sa, int64_t sb,
                                                           int64_t sc) {
  for (int64_t z = (int64_t)blockIdx.x * 256 + threadIdx.x; z < batch; z += (int64_t)gridDim.x * 256) {
    iaat_problem q;
    q.A = P.A + z * sa;
    q.B = P.B + z * sb;
    q.C = P.C + z * sc;
    q.trans = trans;
    q.m = P.m;
    q.n = P.n;
    q.k = P.k;
    q.lda = P.lda;
    q.ldb = P.ldb;
    q.ldc = P.ldc;
    q.alpha = P.alpha;
    q.beta = P.beta;
    q.ab_scale = 1.0f;
    d[z] = q;
  }
}

__global__ __launch_bounds__(64) void scale_strided_kernel(float* C, int m, int n, int ldc, float beta,
                                                           int64_t sc, int64_t batch) {
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y)
    scale_columns(C + z * sc, m, n, ldc, beta, (int)blockIdx.x, (int)gridDim.x);
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
// window counter that hands windows of up to 16 problems out to work-groups.  Each GPU
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
  if (max_blocks < 1) return hipSuccess;
  const dim3 block(64);
  const int64_t nsb = (int64_t)nsm * nsn;
  const int64_t zmax = 0x7fffffffLL / max_blocks;  // grid.x limit
  for (int64_t z0 = 0; z0 < batch; z0 += zmax) {
    const int64_t nz = batch - z0 < zmax ? batch - z0 : zmax;
    dev::Prob Q = P;
    Q.A += z0 * sa;
    Q.B += z0 * sb;
    Q.C += z0 * sc;
    for (int64_t s0 = 0; s0 < nsb; s0 += 65535) {  // grid.y limit
      const int64_t ns = nsb - s0 < 65535 ? nsb - s0 : 65535;
      const dim3 grid((unsigned)(nz * max_blocks), (unsigned)ns, 1);
      const int b0 = (int)s0;
      switch (layout) {
        case 0: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<0, 0>), grid, block, 0, stream, Q, sa, sb, sc, nz, table_dev, nsn, b0, max_blocks); break;
        case 1: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<1, 0>), grid, block, 0, stream, Q, sa, sb, sc, nz, table_dev, nsn, b0, max_blocks); break;
        case 2: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<0, 1>), grid, block, 0, stream, Q, sa, sb, sc, nz, table_dev, nsn, b0, max_blocks); break;
        default: hipLaunchKernelGGL((dev::gemm_f32_strided_kernel<1, 1>), grid, block, 0, stream, Q, sa, sb, sc, nz, table_dev, nsn, b0, max_blocks); break;
      }
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_strided_desc(iaat_problem* d, int64_t batch, const dev::Prob& P, int layout,
                               int64_t sa, int64_t sb, int64_t sc, hipStream_t stream) {
  const int64_t g = (batch + 255) / 256;
  hipLaunchKernelGGL(dev::strided_desc_kernel, dim3((unsigned)(g < 4096 ? g : 4096)), dim3(256), 0, stream, d,
                     batch, P, layout, sa, sb, sc);
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

hipError_t launch_vbatched_f32(const VbArgs& a, int grid, hipStream_t stream) {
  if (a.ticket != nullptr) {
    hipLaunchKernelGGL(dev::clear_ticket_kernel, dim3(1), dim3(64), 0, stream, a.ticket);
    const hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  return launch_vbatched_f32_staged(a, grid, stream);
}

hipError_t vbatched_occupancy(int* blocks_per_cu) { return vbatched_staged_occupancy(blocks_per_cu); }

}  // namespace iaat
