// The traditional small-GEMM scheme, kept as an ablation of IAAT on the GPU
// (the comparison of Section I and Fig. 2(a) with Section V).
//
// Step 1 (pack): op(A) and op(B) of every problem are copied into zero-padded
// tile-contiguous buffers (rows and K rounded up to 16), the extra copy the
// paper measures as the pack step's share of the time.
// Step 2 (compute): one uniform kernel, a 16 x 16 matrix-core tile per
// wavefront over the padded buffers; the padding makes every tile full, so
// only the C store is masked (the boundary handling IAAT's size-specialised
// kernels avoid).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace iaat {
namespace dev {

typedef float f4t __attribute__((ext_vector_type(4)));

// op(A)(i, k) and op(B)(k, j) of a problem.
__device__ __forceinline__ float op_a(const TradProb& P, int i, int k) {
  return (P.trans & 1) ? P.A[k + (int64_t)i * P.lda] : P.A[i + (int64_t)k * P.lda];
}
__device__ __forceinline__ float op_b(const TradProb& P, int k, int j) {
  return (P.trans & 2) ? P.B[j + (int64_t)k * P.ldb] : P.B[k + (int64_t)j * P.ldb];
}

// Packed layout: tile row t (16 rows of op(A)) occupies k16 * 16 floats,
// element (t*16 + r, k) at Ap[(t * k16 + k) * 16 + r]; op(B) likewise by
// tile column, element (k, t*16 + c) at Bp[(t * k16 + k) * 16 + c].
__global__ __launch_bounds__(256) void trad_pack_kernel(const TradProb* probs, int64_t count,
                                                        float* work) {
  for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
    const TradProb P = probs[q];
    float* Ap = work + P.a_off;
    float* Bp = work + P.b_off;
    const int64_t na = (int64_t)P.m16 * P.k16, nb = (int64_t)P.n16 * P.k16;
    for (int64_t e = threadIdx.x; e < na; e += blockDim.x) {
      const int r = (int)(e & 15), kk = (int)((e >> 4) % P.k16), t = (int)((e >> 4) / P.k16);
      const int i = 16 * t + r;
      Ap[e] = (i < P.m && kk < P.k) ? op_a(P, i, kk) : 0.0f;
    }
    for (int64_t e = threadIdx.x; e < nb; e += blockDim.x) {
      const int c = (int)(e & 15), kk = (int)((e >> 4) % P.k16), t = (int)((e >> 4) / P.k16);
      const int j = 16 * t + c;
      Bp[e] = (j < P.n && kk < P.k) ? op_b(P, kk, j) : 0.0f;
    }
  }
}

// One 16 x 16 tile of C per wavefront: tiles[w] = (problem, tile row, tile col).
__global__ __launch_bounds__(64) void trad_tile_kernel(const TradProb* probs, const int32_t* tiles,
                                                       int64_t ntiles, const float* work) {
  const int l = (int)threadIdx.x, r = l & 15, g = l >> 4;
  for (int64_t w = blockIdx.x; w < ntiles; w += gridDim.x) {
    const int32_t q = tiles[3 * w], ti = tiles[3 * w + 1], tj = tiles[3 * w + 2];
    const TradProb P = probs[q];
    const float* Ap = work + P.a_off + (int64_t)ti * P.k16 * 16;
    const float* Bp = work + P.b_off + (int64_t)tj * P.k16 * 16;
    f4t acc = {0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < P.k16; kc += 16) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int kk = kc + 4 * g + s;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Ap[kk * 16 + r], Bp[kk * 16 + r], acc, 0, 0, 0);
      }
    }
    const int j = 16 * tj + r;
    if (j < P.n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * ti + 4 * g + v;
        if (i < P.m) {
          float* c = P.C + i + (int64_t)j * P.ldc;
          *c = P.beta == 0.0f ? P.alpha * acc[v] : fmaf(P.alpha, acc[v], P.beta * *c);
        }
      }
    }
  }
}

}  // namespace dev

hipError_t launch_trad_pack(const TradProb* probs, int64_t count, float* work, int grid,
                            hipStream_t stream) {
  hipLaunchKernelGGL(dev::trad_pack_kernel, dim3((unsigned)grid), dim3(256), 0, stream, probs, count, work);
  return hipGetLastError();
}

hipError_t launch_trad_tiles(const TradProb* probs, const int32_t* tiles, int64_t ntiles,
                             const float* work, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::trad_tile_kernel, dim3((unsigned)grid), dim3(64), 0, stream, probs, tiles,
                     ntiles, work);
  return hipGetLastError();
}

}  // namespace iaat
