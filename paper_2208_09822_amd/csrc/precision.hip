// Reduced-precision inputs for the batched form: on-device quantisation of
// FP32 operands and matrix-core GEMM with FP32 accumulation.
//
// The paper's kernels cover FP32/FP64 real and complex data (Table 1); the
// reduced-precision modes extend the same operation, C = alpha*op(A)*op(B) +
// beta*C with C, alpha, beta and the accumulation in FP32, to A and B held
// as bfloat16, binary16, FP8 E4M3 (OCP, with a per-matrix power-of-two
// scale) or a bfloat16 hi/lo pair (three-product compensation).  Every
// product of two such inputs is exact in FP32, so a result differs from the
// exact product of the dequantised inputs only by FP32 accumulation.
//
// Quantisers are integer bit manipulations of the FP32 pattern, round to
// nearest even, so their codes are fully determined (and checked against the
// format definitions bit for bit).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace iaat {
namespace dev {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef _Float16 h4v __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ quantisers

__device__ __forceinline__ uint32_t fbits(float x) { return __builtin_bit_cast(uint32_t, x); }

// Round-to-nearest-even right shift of a positive integer by `sh` (1..31).
__device__ __forceinline__ uint32_t rne_shift(uint32_t m, int sh) {
  return (m + (1u << (sh - 1)) - 1u + ((m >> sh) & 1u)) >> sh;
}

// bfloat16: the top half of the binary32 pattern, rounded; NaN stays NaN.
__device__ __forceinline__ uint16_t to_bf16(float x) {
  const uint32_t u = fbits(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// IEEE binary16; overflow (|x| >= 65520) gives inf, subnormals have quantum
// 2^-24.
__device__ __forceinline__ uint16_t to_f16(float x) {
  const uint32_t u = fbits(x);
  const uint32_t s = (u >> 16) & 0x8000u, a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint16_t)(s | 0x7e00u | ((a >> 13) & 0x3ffu));
  if (a >= 0x477ff000u) return (uint16_t)(s | 0x7c00u);
  if (a >= 0x38800000u) {  // normal: rebias the exponent 127 -> 15, round off 13 bits
    const uint32_t r = a - 0x38000000u;
    return (uint16_t)(s | ((r + 0x0fffu + ((r >> 13) & 1u)) >> 13));
  }
  const int E = (int)(a >> 23);  // subnormal binary16: code = rint(|x| * 2^24)
  const int sh = 126 - E;
  if (E == 0 || sh > 24) return (uint16_t)s;
  return (uint16_t)(s | rne_shift((a & 0x7fffffu) | 0x800000u, sh));
}

// FP8 E4M3 (OCP "FN" variant: bias 7, no infinities, largest finite 448),
// saturating; -0 is returned as +0 (zero's sign never changes a product).
__device__ __forceinline__ uint8_t to_e4m3(float x) {
  const uint32_t u = fbits(x);
  const uint32_t s = (u >> 24) & 0x80u, a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return (uint8_t)(s | 0x7fu);
  uint32_t c;
  if (a >= 0x43e00000u) {
    c = 0x7eu;  // saturate at 448
  } else if (a >= 0x3c800000u) {  // normal: rebias 127 -> 7, round off 20 bits
    const uint32_t r = a - 0x3c000000u;
    c = (r + 0x7ffffu + ((r >> 20) & 1u)) >> 20;
  } else {  // subnormal E4M3: code = rint(|x| * 2^9)
    const int E = (int)(a >> 23);
    const int sh = 141 - E;
    c = (E == 0 || sh > 24) ? 0u : rne_shift((a & 0x7fffffu) | 0x800000u, sh);
  }
  return (uint8_t)(c == 0 ? 0u : (s | c));
}

// Exponent e of the per-matrix FP8 scale 2^e: the largest e with
// absmax * 2^e <= 448 (448 = 1.75 * 2^8); 0 when absmax is 0 or not finite.
__device__ __forceinline__ int fp8_scale_exp(uint32_t amax_bits) {
  if (amax_bits == 0 || amax_bits >= 0x7f800000u) return 0;
  int E;
  uint32_t frac;
  if (amax_bits >> 23) {
    E = (int)(amax_bits >> 23) - 127;
    frac = amax_bits & 0x7fffffu;
  } else {  // subnormal absmax
    const int p = 31 - __builtin_clz(amax_bits);
    E = p - 149;
    frac = (amax_bits << (23 - p)) & 0x7fffffu;
  }
  return frac <= 0x600000u ? 8 - E : 7 - E;
}

// Largest |x| pattern over n elements, reduced over the work-group.
__device__ uint32_t block_absmax_bits(const float* x, int64_t n, uint32_t* red) {
  uint32_t m = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t a = fbits(x[i]) & 0x7fffffffu;
    m = a > m ? a : m;
  }
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t o = (uint32_t)__shfl_xor((int)m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  uint32_t r = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r = red[w] > r ? red[w] : r;
  __syncthreads();
  return r;
}

// Four 16-bit codes of four floats, 16-byte loads and 8-byte stores where
// source and destination allow it (the encoders run per element either way).
template <class Enc>
__device__ __forceinline__ void encode16(const float* src, uint16_t* d, int64_t n, Enc enc) {
  int64_t i0 = 0;
  if ((((uintptr_t)src & 15) == 0) && (((uintptr_t)d & 7) == 0)) {
    const int64_t n4 = n >> 2;
    const float4* s4 = (const float4*)src;
    uint2* d4 = (uint2*)d;
    for (int64_t i = threadIdx.x; i < n4; i += blockDim.x) {
      const float4 v = s4[i];
      d4[i] = uint2{(uint32_t)enc(v.x) | ((uint32_t)enc(v.y) << 16),
                    (uint32_t)enc(v.z) | ((uint32_t)enc(v.w) << 16)};
    }
    i0 = n4 << 2;
  }
  for (int64_t i = i0 + threadIdx.x; i < n; i += blockDim.x) d[i] = enc(src[i]);
}

// One operand of one job: returns the scale exponent used (FP8) or 0.
__device__ int quantize_operand(int prec, const float* src, void* dst, int64_t n, uint32_t* red) {
  if (n <= 0) return 0;
  if (prec == IAAT_PREC_BF16) {
    encode16(src, (uint16_t*)dst, n, [](float x) { return to_bf16(x); });
    return 0;
  }
  if (prec == IAAT_PREC_F16) {
    encode16(src, (uint16_t*)dst, n, [](float x) { return to_f16(x); });
    return 0;
  }
  if (prec == IAAT_PREC_BF16X3) {  // hi = bf16(x) in [0, n), lo = bf16(x - hi) in [n, 2n)
    uint16_t* d = (uint16_t*)dst;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const float x = src[i];
      const uint16_t hi = to_bf16(x);
      const float hv = __builtin_bit_cast(float, (uint32_t)hi << 16);
      d[i] = hi;
      d[n + i] = to_bf16(x - hv);  // exact in FP32
    }
    return 0;
  }
  // FP8 E4M3 with the power-of-two absmax scale
  const int e = fp8_scale_exp(block_absmax_bits(src, n, red));
  uint8_t* d = (uint8_t*)dst;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) d[i] = to_e4m3(ldexpf(src[i], e));
  return e;
}

__global__ __launch_bounds__(256) void quantize_kernel(int prec, const iaat_qjob* jobs, int64_t count) {
  __shared__ uint32_t red[4];
  for (int64_t j = blockIdx.x; j < count; j += gridDim.x) {
    const iaat_qjob J = jobs[j];
    const int ea = quantize_operand(prec, J.a_src, J.a_dst, J.a_n, red);
    const int eb = quantize_operand(prec, J.b_src, J.b_dst, J.b_n, red);
    if (threadIdx.x == 0) {
      if (J.prob != nullptr) J.prob->ab_scale = ldexpf(1.0f, -(ea + eb));
      if (J.scales != nullptr) {
        J.scales[0] = ldexpf(1.0f, ea);
        J.scales[1] = ldexpf(1.0f, eb);
      }
    }
  }
}

// ------------------------------------------------------------ GEMM

// Element (r, c) of a stored column-major matrix, 0 outside [0, rows) in the
// K direction handled by the caller.
template <typename T>
__device__ __forceinline__ T ld_el(const T* X, int64_t r, int64_t c, int64_t ld) {
  return X[r + c * ld];
}

// Fragment of op(A) for one 16 x 16 tile step: KW consecutive k values of
// row i (with TAIL, k >= K give code 0, which is +0 in every format; full
// chunks skip the test).
template <typename T, int KW, int TA, bool TAIL>
__device__ __forceinline__ void frag_a(const T* A, int64_t lda, int i, int k0, int K, T* out) {
#pragma unroll
  for (int e = 0; e < KW; ++e) {
    const int k = k0 + e;
    if (TAIL)
      out[e] = k < K ? (TA ? ld_el(A, k, i, lda) : ld_el(A, i, k, lda)) : (T)0;
    else
      out[e] = TA ? ld_el(A, k, i, lda) : ld_el(A, i, k, lda);
  }
}
template <typename T, int KW, int TB, bool TAIL>
__device__ __forceinline__ void frag_b(const T* B, int64_t ldb, int j, int k0, int K, T* out) {
#pragma unroll
  for (int e = 0; e < KW; ++e) {
    const int k = k0 + e;
    if (TAIL)
      out[e] = k < K ? (TB ? ld_el(B, j, k, ldb) : ld_el(B, k, j, ldb)) : (T)0;
    else
      out[e] = TB ? ld_el(B, j, k, ldb) : ld_el(B, k, j, ldb);
  }
}

// Exact binary16 pattern of an E4M3 code: every E4M3 value (normal 2^-6 ..
// 448, subnormal m * 2^-9) is a binary16 value.  FP8 operands are multiplied
// as binary16 on the matrix cores: the FP8 matrix-core instruction sums its
// products with fewer bits than FP32 (one scaled unit of a 17-bit exact sum
// was lost in testing), while binary16 products accumulate in FP32.
__device__ __forceinline__ uint16_t e4m3_to_f16(uint8_t c) {
  const uint32_t s = (uint32_t)(c & 0x80u) << 8, a = c & 0x7fu;
  if (a == 0x7fu) return (uint16_t)(s | 0x7e00u);                   // NaN
  if (a >= 0x08u) return (uint16_t)(s | ((a << 7) + 0x2000u));      // normal: rebias 7 -> 15
  if (a == 0) return (uint16_t)s;
  const int p = 31 - __builtin_clz(a);                               // subnormal m * 2^-9
  return (uint16_t)(s | ((uint32_t)(p + 6) << 10) | ((a << (10 - p)) & 0x3ffu));
}

// Products of one 16-wide k-step of a 16 x 16 tile.  Lane l supplies row
// l%16 of op(A) and column l%16 of op(B) at k = k0 + 4*(l/16) + 0..3.
template <int PREC, int TA, int TB, bool TAIL>
__device__ __forceinline__ f4v tile_step(const void* Av, const void* Bv, int64_t lda, int64_t ldb,
                                         int64_t a_lo, int64_t b_lo, int i, int j, int k0, int K,
                                         f4v acc) {
  const int g = (int)(threadIdx.x & 63) >> 4;
  if constexpr (PREC == IAAT_PREC_F8E4M3) {
    uint8_t a[4], b[4];
    frag_a<uint8_t, 4, TA, TAIL>((const uint8_t*)Av, lda, i, k0 + 4 * g, K, a);
    frag_b<uint8_t, 4, TB, TAIL>((const uint8_t*)Bv, ldb, j, k0 + 4 * g, K, b);
    h4v va, vb;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      va[e] = __builtin_bit_cast(_Float16, e4m3_to_f16(a[e]));
      vb[e] = __builtin_bit_cast(_Float16, e4m3_to_f16(b[e]));
    }
    return __builtin_amdgcn_mfma_f32_16x16x16f16(va, vb, acc, 0, 0, 0);
  } else {
    uint16_t a[4], b[4];
    const uint16_t* A = (const uint16_t*)Av;
    const uint16_t* B = (const uint16_t*)Bv;
    frag_a<uint16_t, 4, TA, TAIL>(A, lda, i, k0 + 4 * g, K, a);
    frag_b<uint16_t, 4, TB, TAIL>(B, ldb, j, k0 + 4 * g, K, b);
    if constexpr (PREC == IAAT_PREC_F16) {
      h4v va, vb;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        va[e] = __builtin_bit_cast(_Float16, a[e]);
        vb[e] = __builtin_bit_cast(_Float16, b[e]);
      }
      return __builtin_amdgcn_mfma_f32_16x16x16f16(va, vb, acc, 0, 0, 0);
    } else {
      s4v va, vb;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        va[e] = (short)a[e];
        vb[e] = (short)b[e];
      }
      if constexpr (PREC == IAAT_PREC_BF16X3) {
        // small terms first: lo*hi + hi*lo, then hi*hi
        uint16_t al[4], bl[4];
        frag_a<uint16_t, 4, TA, TAIL>(A + a_lo, lda, i, k0 + 4 * g, K, al);
        frag_b<uint16_t, 4, TB, TAIL>(B + b_lo, ldb, j, k0 + 4 * g, K, bl);
        s4v val, vbl;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          val[e] = (short)al[e];
          vbl[e] = (short)bl[e];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(val, vb, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va, vbl, acc, 0, 0, 0);
      }
      return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(va, vb, acc, 0, 0, 0);
    }
  }
}

// One problem on one wavefront: C is covered by 16 x 16 matrix-core tiles,
// taken in turn; each tile runs the whole K (full 16-wide chunks without a
// K test, then the partial chunk), then the FP32 epilogue.
template <int PREC, int TA, int TB>
__device__ void lowp_problem(const iaat_problem& P) {
  const int KS = 16;
  const int l = (int)(threadIdx.x & 63);
  const int m = P.m, n = P.n, K = P.k;
  const int64_t lda = P.lda, ldb = P.ldb, ldc = P.ldc;
  // the lo halves of split operands follow the hi matrices
  const int64_t a_lo = lda * (TA ? m : K), b_lo = ldb * (TB ? K : n);
  const float alpha = P.alpha * P.ab_scale, beta = P.beta;
  const int tm = (m + 15) >> 4, tn = (n + 15) >> 4;
  const int kfull = K & ~(KS - 1);
  for (int t = 0; t < tm * tn; ++t) {
    const int i0 = 16 * (t % tm), j0 = 16 * (t / tm);
    const int i = min(i0 + (l & 15), m - 1), j = min(j0 + (l & 15), n - 1);
    f4v acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < kfull; k0 += KS)
      acc = tile_step<PREC, TA, TB, false>(P.A, P.B, lda, ldb, a_lo, b_lo, i, j, k0, K, acc);
    if (kfull < K)
      acc = tile_step<PREC, TA, TB, true>(P.A, P.B, lda, ldb, a_lo, b_lo, i, j, kfull, K, acc);
    const int jc = j0 + (l & 15);
    if (jc < n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ic = i0 + 4 * (l >> 4) + v;
        if (ic < m) {
          float* c = P.C + ic + jc * ldc;
          *c = beta == 0.0f ? alpha * acc[v] : fmaf(alpha, acc[v], beta * *c);
        }
      }
    }
  }
}

// Wavefront w of the grid (four per work-group) takes problems w, w + W, ...
// (W wavefronts in all): small problems keep every wavefront busy.  The FP8
// kernel is held to eight wavefronts per SIMD (a few spills; its widening
// of the codes adds latency that more wavefronts hide); for the others more
// wavefronts per SIMD measured slower.
template <int PREC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == IAAT_PREC_F8E4M3 ? 8 : 1)))
void vbatched_lowp_kernel(VbArgs a) {
  const int64_t W = (int64_t)gridDim.x * 4;
  const int64_t w0 = (int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int l = (int)(threadIdx.x & 63);
  for (int64_t q = w0; q < a.count; q += W) {
    const iaat_problem P = a.probs[q];
    const int st = validate(P.trans, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, P.alpha, P.A, P.B, P.C);
    if (l == 0 && a.status != nullptr) a.status[q] = st;
    if (st != 0 || P.m == 0 || P.n == 0) continue;
    if (P.alpha == 0.0f || P.k == 0) {  // C = beta*C, A and B not read
      for (int64_t e = l; e < (int64_t)P.m * P.n; e += 64) {
        float* c = P.C + e % P.m + (e / P.m) * (int64_t)P.ldc;
        *c = P.beta == 0.0f ? 0.0f : P.beta * *c;
      }
      continue;
    }
    switch (P.trans) {
      case 0: lowp_problem<PREC, 0, 0>(P); break;
      case 1: lowp_problem<PREC, 1, 0>(P); break;
      case 2: lowp_problem<PREC, 0, 1>(P); break;
      default: lowp_problem<PREC, 1, 1>(P); break;
    }
  }
}

}  // namespace dev

hipError_t launch_quantize(int prec, const iaat_qjob* jobs, int64_t count, int grid, hipStream_t stream) {
  hipLaunchKernelGGL(dev::quantize_kernel, dim3((unsigned)grid), dim3(256), 0, stream, prec, jobs, count);
  return hipGetLastError();
}

hipError_t launch_vbatched_lowp(const VbArgs& a, int prec, int grid, hipStream_t stream) {
  switch (prec) {
    case IAAT_PREC_BF16:
      hipLaunchKernelGGL(dev::vbatched_lowp_kernel<IAAT_PREC_BF16>, dim3((unsigned)grid), dim3(256), 0, stream, a);
      break;
    case IAAT_PREC_F16:
      hipLaunchKernelGGL(dev::vbatched_lowp_kernel<IAAT_PREC_F16>, dim3((unsigned)grid), dim3(256), 0, stream, a);
      break;
    case IAAT_PREC_F8E4M3:
      hipLaunchKernelGGL(dev::vbatched_lowp_kernel<IAAT_PREC_F8E4M3>, dim3((unsigned)grid), dim3(256), 0, stream, a);
      break;
    default:
      hipLaunchKernelGGL(dev::vbatched_lowp_kernel<IAAT_PREC_BF16X3>, dim3((unsigned)grid), dim3(256), 0, stream, a);
      break;
  }
  return hipGetLastError();
}

}  // namespace iaat
