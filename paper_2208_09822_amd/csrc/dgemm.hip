// DGEMM (Table 1, row D): C = alpha*op(A)*op(B) + beta*C in FP64 on the
// matrix cores (v_mfma_f64_16x16x4_f64).
//
// Lane l supplies op(A)(row l%16, k-slot l/16) and op(B)(k-slot l/16,
// col l%16); its four results are rows l/16 + 4v (v = 0..3) of column l%16
// (unlike the FP32 instruction's rows 4(l/16) + v).
// The M x N of C is covered by 16 x 16 tiles, grouped into blocks of at most
// 3 x 3 tiles, the groups per dimension as even as possible (the grouping
// rule of the FP32 tiler's matrix-core plans); one wavefront computes one
// block, reading A and B in place with the rows and columns past the edge
// clamped (never stored) and the K tail zero-filled -- no pack, no boundary
// kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace iaat {
namespace dev {

typedef double d4 __attribute__((ext_vector_type(4)));

// Start and size of group g when t tiles are split into ng groups.
__device__ __forceinline__ void tile_group(int t, int ng, int g, int& start, int& size) {
  const int q = t / ng, r = t % ng;
  size = q + (g < r ? 1 : 0);
  start = g * q + (g < r ? g : r);
}

template <int TA, int TB>
__device__ __forceinline__ void dgemm_block(const DProb& P, int bi, int bj) {
  const int l = (int)(threadIdx.x & 63), r = l & 15, g = l >> 4;
  const int tm = (P.m + 15) >> 4, tn = (P.n + 15) >> 4;
  const int gm = (tm + 2) / 3, gn = (tn + 2) / 3;
  int r0, TM, c0, TN;
  tile_group(tm, gm, bi, r0, TM);
  tile_group(tn, gn, bj, c0, TN);
  int ia[3], jb[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    ia[t] = min(16 * (r0 + t) + r, P.m - 1);
    jb[t] = min(16 * (c0 + t) + r, P.n - 1);
  }
  d4 acc[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t lda = P.lda, ldb = P.ldb;
  for (int kc = 0; kc < P.k; kc += 4) {
    const int k = kc + g;
    const bool ok = k < P.k;
    const int kk = ok ? k : P.k - 1;
    double av[3], bv[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const double x = TA ? P.A[kk + ia[t] * lda] : P.A[ia[t] + kk * lda];
      const double y = TB ? P.B[jb[t] + kk * ldb] : P.B[kk + jb[t] * ldb];
      av[t] = ok ? x : 0.0;
      bv[t] = ok ? y : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        if (a < TM && b < TN) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
  }
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int j = 16 * (c0 + b) + r;
    if (b >= TN || j >= P.n) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= TM) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * (r0 + a) + g + 4 * v;  // the FP64 result layout: row g + 4v
        if (i < P.m) {
          double* c = P.C + i + (int64_t)j * P.ldc;
          *c = P.beta == 0.0 ? P.alpha * acc[a][b][v] : fma(P.alpha, acc[a][b][v], P.beta * *c);
        }
      }
    }
  }
}

// grid: x = block (bi * gn + bj), y = problem z (grid-stride), one wavefront each.
template <int TA, int TB>
__global__ __launch_bounds__(64) void dgemm_kernel(DProb P, int64_t sa, int64_t sb, int64_t sc,
                                                   int64_t batch, int gn) {
  const int bi = (int)blockIdx.x / gn, bj = (int)blockIdx.x - bi * gn;
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y) {
    DProb Q = P;
    Q.A += z * sa;
    Q.B += z * sb;
    Q.C += z * sc;
    dgemm_block<TA, TB>(Q, bi, bj);
  }
}

// C = beta*C for every problem (alpha == 0 or K == 0).
__global__ __launch_bounds__(256) void dscale_kernel(double* C, int m, int n, int64_t ldc, double beta,
                                                     int64_t sc, int64_t batch) {
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y)
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < (int64_t)m * n; e += (int64_t)gridDim.x * 256) {
      double* c = C + z * sc + e % m + (e / m) * ldc;
      *c = beta == 0.0 ? 0.0 : beta * *c;
    }
}

}  // namespace dev

hipError_t launch_dgemm(const DProb& P, int layout, int64_t sa, int64_t sb, int64_t sc, int64_t batch,
                        hipStream_t stream) {
  const int tm = (P.m + 15) / 16, tn = (P.n + 15) / 16;
  const int gm = (tm + 2) / 3, gn = (tn + 2) / 3;
  const dim3 grid((unsigned)(gm * gn), (unsigned)(batch < 65535 ? batch : 65535)), block(64);
  switch (layout) {
    case 0: hipLaunchKernelGGL((dev::dgemm_kernel<0, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    case 1: hipLaunchKernelGGL((dev::dgemm_kernel<1, 0>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    case 2: hipLaunchKernelGGL((dev::dgemm_kernel<0, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
    default: hipLaunchKernelGGL((dev::dgemm_kernel<1, 1>), grid, block, 0, stream, P, sa, sb, sc, batch, gn); break;
  }
  return hipGetLastError();
}

hipError_t launch_dscale(double* C, int m, int n, int64_t ldc, double beta, int64_t sc, int64_t batch,
                         hipStream_t stream) {
  const int64_t el = (int64_t)m * n;
  const unsigned gx = (unsigned)((el + 255) / 256 < 256 ? (el + 255) / 256 : 256);
  hipLaunchKernelGGL(dev::dscale_kernel, dim3(gx, (unsigned)(batch < 65535 ? batch : 65535)), dim3(256), 0,
                     stream, C, m, n, ldc, beta, sc, batch);
  return hipGetLastError();
}

}  // namespace iaat
