// CGEMM (Table 1, row C): C = alpha*op(A)*op(B) + beta*C with complex
// single-precision operands stored as interleaved (re, im) pairs, complex
// alpha and beta, op(X) = X or X^T.
//
// Same blocking as the real matrix-core path: C's 16 x 16 tiles grouped into
// blocks of at most 3 x 3 tiles, one wavefront per block, operands read in
// place (edges clamped, K tail zero-filled).  A complex product is four
// real v_mfma_f32_16x16x4_f32 accumulations into a real and an imaginary
// accumulator: re += ar*br - ai*bi, im += ar*bi + ai*br.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace iaat {
namespace dev {

typedef float c4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void ctile_group(int t, int ng, int g, int& start, int& size) {
  const int q = t / ng, r = t % ng;
  size = q + (g < r ? 1 : 0);
  start = g * q + (g < r ? g : r);
}

template <int TA, int TB>
__device__ __forceinline__ void cgemm_block(const CProb& P, int bi, int bj) {
  const int l = (int)(threadIdx.x & 63), r = l & 15, g = l >> 4;
  const int tm = (P.m + 15) >> 4, tn = (P.n + 15) >> 4;
  const int gm = (tm + 2) / 3, gn = (tn + 2) / 3;
  int r0, TM, c0, TN;
  ctile_group(tm, gm, bi, r0, TM);
  ctile_group(tn, gn, bj, c0, TN);
  int ia[3], jb[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    ia[t] = min(16 * (r0 + t) + r, P.m - 1);
    jb[t] = min(16 * (c0 + t) + r, P.n - 1);
  }
  c4 re[3][3], im[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      re[a][b] = c4{0.f, 0.f, 0.f, 0.f};
      im[a][b] = c4{0.f, 0.f, 0.f, 0.f};
    }
  const int64_t lda = P.lda, ldb = P.ldb;
  const float2* A = (const float2*)P.A;
  const float2* B = (const float2*)P.B;
  for (int kc = 0; kc < P.k; kc += 4) {
    const int k = kc + g;
    const bool ok = k < P.k;
    const int kk = ok ? k : P.k - 1;
    float2 av[3], bv[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const float2 x = TA ? A[kk + ia[t] * lda] : A[ia[t] + kk * lda];
      const float2 y = TB ? B[jb[t] + kk * ldb] : B[kk + jb[t] * ldb];
      av[t] = ok ? x : float2{0.f, 0.f};
      bv[t] = ok ? y : float2{0.f, 0.f};
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (a < TM && b < TN) {
          re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].x, re[a][b], 0, 0, 0);
          re[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(-av[a].y, bv[b].y, re[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].x, bv[b].y, im[a][b], 0, 0, 0);
          im[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a].y, bv[b].x, im[a][b], 0, 0, 0);
        }
  }
  const bool beta0 = P.beta_re == 0.0f && P.beta_im == 0.0f;
  float2* C = (float2*)P.C;
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int j = 16 * (c0 + b) + r;
    if (b >= TN || j >= P.n) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= TM) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (r0 + a) + 4 * g + v;  // FP32 result layout: rows 4(l/16) + v
        if (i < P.m) {
          float2* c = C + i + (int64_t)j * P.ldc;
          const float sr = re[a][b][v], si = im[a][b][v];
          float xr = P.alpha_re * sr - P.alpha_im * si;
          float xi = P.alpha_re * si + P.alpha_im * sr;
          if (!beta0) {
            const float2 c0v = *c;
            xr += P.beta_re * c0v.x - P.beta_im * c0v.y;
            xi += P.beta_re * c0v.y + P.beta_im * c0v.x;
          }
          *c = float2{xr, xi};
        }
      }
    }
  }
}

template <int TA, int TB>
__global__ __launch_bounds__(64) void cgemm_kernel(CProb P, int64_t sa, int64_t sb, int64_t sc,
                                                   int64_t batch, int gn) {
  const int bi = (int)blockIdx.x / gn, bj = (int)blockIdx.x - bi * gn;
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y) {
    CProb Q = P;
    Q.A += 2 * z * sa;
    Q.B += 2 * z * sb;
    Q.C += 2 * z * sc;
    cgemm_block<TA, TB>(Q, bi, bj);
  }
}

// C = beta*C (alpha == 0 or K == 0), complex beta.
__global__ __launch_bounds__(256) void cscale_kernel(float* C, int m, int n, int64_t ldc, float br,
                                                     float bim, int64_t sc, int64_t batch) {
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y)
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < (int64_t)m * n; e += (int64_t)gridDim.x * 256) {
      float2* c = (float2*)C + z * sc + e % m + (e / m) * ldc;
      if (br == 0.0f && bim == 0.0f) {
        *c = float2{0.f, 0.f};
      } else {
        const float2 v = *c;
        *c = float2{br * v.x - bim * v.y, br * v.y + bim * v.x};
      }
    }
}

}  // namespace dev

hipError_t launch_cgemm(const CProb& P, int layout, int64_t sa, int64_t sb, int64_t sc, int64_t batch,
                        hipStream_t stream) {
  const int tm = (P.m + 15) / 16, tn = (P.n + 15) / 16;
  const int gm = (tm + 2) / 3, gn = (tn + 2) / 3;
  const dim3 grid((unsigned)(gm * gn), (unsigned)(batch < 65535 ? batch : 65535)), block(64);
  switch (layout) {
    case 0: hipLaunchKernelGGL((dev::cgemm_kernel<0, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    case 1: hipLaunchKernelGGL((dev::cgemm_kernel<1, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    case 2: hipLaunchKernelGGL((dev::cgemm_kernel<0, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    default: hipLaunchKernelGGL((dev::cgemm_kernel<1, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
  }
  return hipGetLastError();
}

hipError_t launch_cscale(float* C, int m, int n, int64_t ldc, float beta_re, float beta_im, int64_t sc,
                         int64_t batch, hipStream_t stream) {
  const int64_t el = (int64_t)m * n;
  const unsigned gx = (unsigned)((el + 255) / 256 < 256 ? (el + 255) / 256 : 256);
  hipLaunchKernelGGL(dev::cscale_kernel, dim3(gx, (unsigned)(batch < 65535 ? batch : 65535)), dim3(256), 0,
                     stream, C, m, n, ldc, beta_re, beta_im, sc, batch);
  return hipGetLastError();
}

}  // namespace iaat
