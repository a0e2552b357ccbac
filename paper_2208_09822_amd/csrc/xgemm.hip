// DGEMM, CGEMM and ZGEMM (Table 1, rows D, C and Z) on the input-aware
// path: the run-time tiler's plan for (layout, M, N) -- the same tile table
// the FP32 path uses, since a plan depends on the shape and layout only --
// and each plan block run by the generated family's member for that block
// shape, instantiated for the element type (the family is generated per
// shape, layout and data type).  Operands are read in place (no pack); the
// rows and columns past an edge are clamped and never stored, the K tail is
// zero-filled.
//
//   D  FP64 real: v_mfma_f64_16x16x4_f64 for matrix-core blocks.
//   C  FP32 complex (interleaved re, im): four v_mfma_f32_16x16x4_f32 per
//      complex step, re += ar*br - ai*bi and im += ar*bi + ai*br (Eq. 2).
//   Z  FP64 complex: the same four-product expansion on the FP64 matrix
//      cores.
// Strip and K-split blocks run FMA chains over K in increasing order (a
// complex product as the same four real products).
//
// Forms: one problem (one work-group per plan block), same-size strided
// batches, and uneven batches described by iaat_xproblem descriptors (one
// wavefront per problem, every block of its plan).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "iaat_internal.h"
#include "kernels.h"

namespace iaat {
namespace dev {


typedef float xf4 __attribute__((ext_vector_type(4)));
typedef double xd4 __attribute__((ext_vector_type(4)));

// Element traits: R is the real type; CPLX whether elements are (re, im).
template <int DT>
struct XT;
template <>
struct XT<IAAT_DT_F64> {
  typedef double R;
  typedef xd4 V;
  static constexpr bool CPLX = false;
};
template <>
struct XT<IAAT_DT_C64> {
  typedef float R;
  typedef xf4 V;
  static constexpr bool CPLX = true;
};
template <>
struct XT<IAAT_DT_C128> {
  typedef double R;
  typedef xd4 V;
  static constexpr bool CPLX = true;
};

template <class R>
struct Cx {
  R re, im;
};

// Element idx of a stored matrix (complex: the pair at 2*idx).
template <int DT>
__device__ __forceinline__ Cx<typename XT<DT>::R> xload(const void* X, int64_t idx) {
  typedef typename XT<DT>::R R;
  const R* p = (const R*)X;
  if (XT<DT>::CPLX) return Cx<R>{p[2 * idx], p[2 * idx + 1]};
  return Cx<R>{p[idx], (R)0};
}

template <int DT>
__device__ __forceinline__ void xstore(void* X, int64_t idx, Cx<typename XT<DT>::R> v) {
  typedef typename XT<DT>::R R;
  R* p = (R*)X;
  if (XT<DT>::CPLX) {
    p[2 * idx] = v.re;
    p[2 * idx + 1] = v.im;
  } else {
    p[idx] = v.re;
  }
}

// op(A)(i, p) and op(B)(p, j) as element indices of the stored matrices.
template <int TA>
__device__ __forceinline__ int64_t aidx(const XProb& P, int i, int p) {
  return TA ? (int64_t)p + (int64_t)i * P.lda : (int64_t)i + (int64_t)p * P.lda;
}
template <int TB>
__device__ __forceinline__ int64_t bidx(const XProb& P, int p, int j) {
  return TB ? (int64_t)j + (int64_t)p * P.ldb : (int64_t)p + (int64_t)j * P.ldb;
}

// The epilogue: alpha*s + beta*C (C not read when beta == 0).
template <int DT>
__device__ __forceinline__ Cx<typename XT<DT>::R> xepi(const XProb& P, Cx<typename XT<DT>::R> s,
                                                      int64_t ci) {
  typedef typename XT<DT>::R R;
  const R ar = (R)P.alpha_re, ai = (R)P.alpha_im, br = (R)P.beta_re, bi = (R)P.beta_im;
  Cx<R> o;
  if (!XT<DT>::CPLX) {
    o.re = br == (R)0 ? ar * s.re : fma(ar, s.re, br * xload<DT>(P.C, ci).re);
    o.im = (R)0;
    return o;
  }
  o.re = ar * s.re - ai * s.im;
  o.im = ar * s.im + ai * s.re;
  if (br != (R)0 || bi != (R)0) {
    const Cx<R> c = xload<DT>(P.C, ci);
    o.re += br * c.re - bi * c.im;
    o.im += br * c.im + bi * c.re;
  }
  return o;
}

__device__ __forceinline__ xf4 xmfma(float a, float b, xf4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ xd4 xmfma(double a, double b, xd4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// Row (within a 16 x 16 tile) of result v of lane group g: FP32 rows
// 4g + v, FP64 rows g + 4v.
template <class R>
__device__ __forceinline__ int xrow(int g, int v) {
  return sizeof(R) == 4 ? 4 * g + v : g + 4 * v;
}

// TM x TN (<= 3 x 3) grid of 16 x 16 matrix-core tiles at (i0, j0).  Step
// kc of K gives lane group g = l/16 the reduction index kc + g.
template <int DT, int TA, int TB, int TM, int TN>
struct XMfma {
  static __device__ __forceinline__ void run(const XProb& P, int i0, int j0) {
    typedef typename XT<DT>::R R;
    typedef typename XT<DT>::V V;
    const int l = (int)(threadIdx.x & 63), r = l & 15, g = l >> 4;
    int ia[TM], jb[TN];
#pragma unroll
    for (int t = 0; t < TM; ++t) ia[t] = min(i0 + 16 * t + r, P.m - 1);
#pragma unroll
    for (int t = 0; t < TN; ++t) jb[t] = min(j0 + 16 * t + r, P.n - 1);
    V re[TM][TN], im[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        re[a][b] = V{0, 0, 0, 0};
        im[a][b] = V{0, 0, 0, 0};
      }
#pragma unroll 2
    for (int kc = 0; kc < P.k; kc += 4) {
      const int k = kc + g;
      const bool ok = k < P.k;
      const int kk = ok ? k : P.k - 1;
      Cx<R> av[TM], bv[TN];
#pragma unroll
      for (int t = 0; t < TM; ++t) {
        const Cx<R> x = xload<DT>(P.A, aidx<TA>(P, ia[t], kk));
        av[t] = ok ? x : Cx<R>{(R)0, (R)0};
      }
#pragma unroll
      for (int t = 0; t < TN; ++t) {
        const Cx<R> y = xload<DT>(P.B, bidx<TB>(P, kk, jb[t]));
        bv[t] = ok ? y : Cx<R>{(R)0, (R)0};
      }
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
          re[a][b] = xmfma(av[a].re, bv[b].re, re[a][b]);
          if (XT<DT>::CPLX) {
            re[a][b] = xmfma(-av[a].im, bv[b].im, re[a][b]);
            im[a][b] = xmfma(av[a].re, bv[b].im, im[a][b]);
            im[a][b] = xmfma(av[a].im, bv[b].re, im[a][b]);
          }
        }
    }
#pragma unroll
    for (int b = 0; b < TN; ++b) {
      const int j = j0 + 16 * b + r;
      if (j >= P.n) continue;
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = i0 + 16 * a + xrow<R>(g, v);
          if (i >= P.m) continue;
          const int64_t ci = (int64_t)i + (int64_t)j * P.ldc;
          xstore<DT>(P.C, ci, xepi<DT>(P, Cx<R>{re[a][b][v], im[a][b][v]}, ci));
        }
    }
  }
};

template <class R>
__device__ __forceinline__ void cfma(Cx<R>& acc, Cx<R> a, Cx<R> b, bool cplx) {
  acc.re = fma(a.re, b.re, acc.re);
  if (cplx) {
    acc.re = fma(-a.im, b.im, acc.re);
    acc.im = fma(a.re, b.im, acc.im);
    acc.im = fma(a.im, b.re, acc.im);
  }
}

// MR rows x 64 columns, lane = column; FMA chains over K in order.
template <int DT, int TA, int TB, int MR>
struct XRows {
  static __device__ __forceinline__ void run(const XProb& P, int i0, int j0) {
    typedef typename XT<DT>::R R;
    const int j = j0 + (int)(threadIdx.x & 63);
    const int jc = min(j, P.n - 1);
    Cx<R> acc[MR];
#pragma unroll
    for (int i = 0; i < MR; ++i) acc[i] = Cx<R>{(R)0, (R)0};
    for (int p = 0; p < P.k; ++p) {
      const Cx<R> b = xload<DT>(P.B, bidx<TB>(P, p, jc));
#pragma unroll
      for (int i = 0; i < MR; ++i)
        cfma(acc[i], xload<DT>(P.A, aidx<TA>(P, min(i0 + i, P.m - 1), p)), b, XT<DT>::CPLX);
    }
    if (j >= P.n) return;
#pragma unroll
    for (int i = 0; i < MR; ++i) {
      if (i0 + i >= P.m) continue;
      const int64_t ci = (int64_t)(i0 + i) + (int64_t)j * P.ldc;
      xstore<DT>(P.C, ci, xepi<DT>(P, acc[i], ci));
    }
  }
};

// 64 rows x NR columns, lane = row.
template <int DT, int TA, int TB, int NR>
struct XCols {
  static __device__ __forceinline__ void run(const XProb& P, int i0, int j0) {
    typedef typename XT<DT>::R R;
    const int i = i0 + (int)(threadIdx.x & 63);
    const int ic = min(i, P.m - 1);
    Cx<R> acc[NR];
#pragma unroll
    for (int j = 0; j < NR; ++j) acc[j] = Cx<R>{(R)0, (R)0};
    for (int p = 0; p < P.k; ++p) {
      const Cx<R> a = xload<DT>(P.A, aidx<TA>(P, ic, p));
#pragma unroll
      for (int j = 0; j < NR; ++j)
        cfma(acc[j], a, xload<DT>(P.B, bidx<TB>(P, p, min(j0 + j, P.n - 1))), XT<DT>::CPLX);
    }
    if (i >= P.m) return;
#pragma unroll
    for (int j = 0; j < NR; ++j) {
      if (j0 + j >= P.n) continue;
      const int64_t ci = (int64_t)i + (int64_t)(j0 + j) * P.ldc;
      xstore<DT>(P.C, ci, xepi<DT>(P, acc[j], ci));
    }
  }
};

template <class R>
__device__ __forceinline__ R xshfl(R v, int m) {
  if (sizeof(R) == 4) return __shfl_xor(v, m, 64);
  return __shfl_xor(v, m, 64);
}

// MR x NR (<= 4 x 4) block, K split over the lanes (lane l sums k = l,
// l + 64, ...), a butterfly adds the 64 partial sums, lane 0 stores.
template <int DT, int TA, int TB, int MR, int NR>
struct XKred {
  static __device__ __forceinline__ void run(const XProb& P, int i0, int j0) {
    typedef typename XT<DT>::R R;
    const int l = (int)(threadIdx.x & 63);
    Cx<R> acc[MR][NR];
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j) acc[i][j] = Cx<R>{(R)0, (R)0};
    for (int p = l; p < P.k; p += 64) {
      Cx<R> a[MR], b[NR];
#pragma unroll
      for (int i = 0; i < MR; ++i) a[i] = xload<DT>(P.A, aidx<TA>(P, min(i0 + i, P.m - 1), p));
#pragma unroll
      for (int j = 0; j < NR; ++j) b[j] = xload<DT>(P.B, bidx<TB>(P, p, min(j0 + j, P.n - 1)));
#pragma unroll
      for (int i = 0; i < MR; ++i)
#pragma unroll
        for (int j = 0; j < NR; ++j) cfma(acc[i][j], a[i], b[j], XT<DT>::CPLX);
    }
#pragma unroll
    for (int i = 0; i < MR; ++i)
#pragma unroll
      for (int j = 0; j < NR; ++j)
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          acc[i][j].re += xshfl(acc[i][j].re, off);
          if (XT<DT>::CPLX) acc[i][j].im += xshfl(acc[i][j].im, off);
        }
    if (l != 0) return;
#pragma unroll
    for (int j = 0; j < NR; ++j)
#pragma unroll
      for (int i = 0; i < MR; ++i) {
        if (i0 + i >= P.m || j0 + j >= P.n) continue;
        const int64_t ci = (int64_t)(i0 + i) + (int64_t)(j0 + j) * P.ldc;
        xstore<DT>(P.C, ci, xepi<DT>(P, acc[i][j], ci));
      }
  }
};

// The family member for (family, p1, p2) at element type DT.
template <int FAM, int DT, int TA, int TB, int P1, int P2>
struct XBlock;
// Complex grids run one tile row at a time (the register footprint of a
// whole 3 x 3 grid of complex accumulators would cut occupancy to one
// wavefront per SIMD); each tile's arithmetic is unchanged.
template <int DT, int TA, int TB, int P1, int P2>
struct XBlock<0, DT, TA, TB, P1, P2> {
  static __device__ __forceinline__ void run(const XProb& P, int i0, int j0) {
    if (XT<DT>::CPLX) {
      for (int a = 0; a < P1; ++a) XMfma<DT, TA, TB, 1, P2>::run(P, i0 + 16 * a, j0);
    } else {
      XMfma<DT, TA, TB, P1, P2>::run(P, i0, j0);
    }
  }
};
template <int DT, int TA, int TB, int P1, int P2>
struct XBlock<1, DT, TA, TB, P1, P2> : XRows<DT, TA, TB, P1> {};
template <int DT, int TA, int TB, int P1, int P2>
struct XBlock<2, DT, TA, TB, P1, P2> : XCols<DT, TA, TB, P2> {};
template <int DT, int TA, int TB, int P1, int P2>
struct XBlock<3, DT, TA, TB, P1, P2> : XKred<DT, TA, TB, P1, P2> {};

// LIGHT: only the members kid_light() accepts are compiled in (the others
// are never dispatched to such a kernel).
template <int DT, int TA, int TB, bool LIGHT = false>
__device__ __forceinline__ void xrun_block(int kid, const XProb& P, int i0, int j0) {
  switch (kid) {
#define IAAT_XCASE(id, fam, p1, p2, br, bc)                                       \
  case id:                                                                        \
    if constexpr (!LIGHT || kid_light(fam, p1, p2, XT<DT>::CPLX)) XBlock<fam, DT, TA, TB, p1, p2>::run(P, i0, j0); \
    break;
    IAAT_FOR_EACH_KID(IAAT_XCASE)
#undef IAAT_XCASE
    default:
      break;
  }
}

// Super-block (sbi, sbj): rows and columns [80 s, 80 s + 80) of C.
template <int DT, int TA, int TB>
__device__ __forceinline__ XProb xsub(const XProb& P, int sbi, int sbj) {
  const int64_t es = XT<DT>::CPLX ? 2 * (int64_t)sizeof(typename XT<DT>::R)
                                  : (int64_t)sizeof(typename XT<DT>::R);
  const int64_t r0 = (int64_t)sbi * kSuper, c0 = (int64_t)sbj * kSuper;
  XProb S = P;
  S.A = (const char*)P.A + es * (TA ? r0 * P.lda : r0);
  S.B = (const char*)P.B + es * (TB ? c0 : c0 * P.ldb);
  S.C = (char*)P.C + es * (r0 + c0 * P.ldc);
  S.m = (int)min((int64_t)kSuper, (int64_t)P.m - r0);
  S.n = (int)min((int64_t)kSuper, (int64_t)P.n - c0);
  return S;
}

// One problem (or a same-size strided batch): one plan block of one
// super-block of one problem per work-group (the host launches very long
// batches and very many super-blocks in pieces).  The register
// budget is that of the largest member compiled in: LIGHT kernels run eight
// wavefronts per SIMD, full kernels four (complex FP64 with a few spills).
template <int DT, int TA, int TB, bool LIGHT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(LIGHT ? 8 : 4)))
void xgemm_kernel(XProb P, int64_t sa, int64_t sb, int64_t sc, int64_t batch,
                  const PlanEntry* __restrict__ table, int nsn, int sb0, int slots) {
  // grid.x = problem * slots + block slot (a problem's blocks run side by
  // side, sharing its operands in cache), grid.y = super-block - sb0
  const int sbk = sb0 + (int)blockIdx.y, b = (int)(blockIdx.x % (unsigned)slots);
  const int64_t z = blockIdx.x / (unsigned)slots;
  const int sbi = sbk / nsn, sbj = sbk - sbi * nsn;
  const int64_t es = XT<DT>::CPLX ? 2 * (int64_t)sizeof(typename XT<DT>::R)
                                  : (int64_t)sizeof(typename XT<DT>::R);
  const XProb S0 = xsub<DT, TA, TB>(P, sbi, sbj);
  const PlanEntry* e = table + plan_index(TA | (TB << 1), S0.m, S0.n);
  if (b >= (int)e->nblk) return;
  const uint32_t w = e->blk[b];
  // one block of one problem per work-group (no loop over the batch: a loop
  // around the member switch more than doubled the registers it takes)
  if (z >= batch) return;
  XProb Q = S0;
  Q.A = (const char*)S0.A + es * z * sa;
  Q.B = (const char*)S0.B + es * z * sb;
  Q.C = (char*)S0.C + es * z * sc;
  xrun_block<DT, TA, TB, LIGHT>(blk_kid(w), Q, blk_i0(w), blk_j0(w));
}

// C = beta*C (alpha == 0 or K == 0), batch along grid.y.
template <int DT>
__global__ __launch_bounds__(256) void xscale_kernel(XProb P, int64_t sc, int64_t batch) {
  typedef typename XT<DT>::R R;
  const int64_t es = XT<DT>::CPLX ? 2 : 1;
  const int64_t mn = (int64_t)P.m * P.n;
  for (int64_t z = blockIdx.y; z < batch; z += gridDim.y)
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < mn; e += (int64_t)gridDim.x * 256) {
      const int64_t ci = e % P.m + (e / P.m) * P.ldc;
      R* c = (R*)P.C + es * z * sc;
      const R br = (R)P.beta_re, bi = (R)P.beta_im;
      if (br == (R)0 && bi == (R)0) {
        xstore<DT>(c, ci, Cx<R>{(R)0, (R)0});
      } else {
        const Cx<R> v = xload<DT>(c, ci);
        xstore<DT>(c, ci, Cx<R>{br * v.re - bi * v.im, br * v.im + bi * v.re});
      }
    }
}

// A whole problem on one wavefront: every super-block, every plan block.
// Inlined, so the kernel's register budget applies to it (an out-of-line
// copy took 248 registers whatever the kernel asked for).
template <int DT, int TA, int TB>
__device__ __forceinline__ void xsolve(XProb P, const PlanEntry* table) {
  const int nsm = (P.m + kSuper - 1) / kSuper, nsn = (P.n + kSuper - 1) / kSuper;
  for (int sbj = 0; sbj < nsn; ++sbj)
    for (int sbi = 0; sbi < nsm; ++sbi) {
      const XProb S = xsub<DT, TA, TB>(P, sbi, sbj);
      const PlanEntry* e = table + plan_index(TA | (TB << 1), S.m, S.n);
      const int nb = (int)e->nblk;
      for (int b = 0; b < nb; ++b) {
        const uint32_t w = e->blk[b];
        xrun_block<DT, TA, TB>(blk_kid(w), S, blk_i0(w), blk_j0(w));
      }
    }
}

__device__ __forceinline__ int xuni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double xunid(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t lo = (uint32_t)xuni((int)(uint32_t)u), hi = (uint32_t)xuni((int)(u >> 32));
  return __builtin_bit_cast(double, lo | (hi << 32));
}
__device__ __forceinline__ const void* xunip(const void* p) {
  const uint64_t v = (uint64_t)p;
  return (const void*)(((uint64_t)(uint32_t)xuni((int)(v >> 32)) << 32) | (uint32_t)xuni((int)v));
}

// Uneven batch: wavefront q of the grid (grid-stride) takes problem q,
// writes its status, and computes it (quick return: C = beta*C).  Every
// member is compiled in; the register budget (no spills) allows five
// wavefronts per SIMD for complex FP32, four for FP64 and three for complex
// FP64 (four, with spills, measured slower).
template <int DT>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(DT == IAAT_DT_C64 ? 5 : DT == IAAT_DT_C128 ? 3 : 4)))
void xgemm_vbatched_kernel(const iaat_xproblem* __restrict__ probs,
                                                            int64_t count, int32_t* status,
                                                            const PlanEntry* __restrict__ table) {
  typedef typename XT<DT>::R R;
  for (int64_t q = blockIdx.x; q < count; q += gridDim.x) {
    const iaat_xproblem& d = probs[q];
    XProb P;
    P.A = xunip(d.A);
    P.B = xunip(d.B);
    P.C = (void*)xunip(d.C);
    const int trans = xuni(d.trans);
    P.m = xuni(d.m);
    P.n = xuni(d.n);
    P.k = xuni(d.k);
    P.lda = xuni(d.lda);
    P.ldb = xuni(d.ldb);
    P.ldc = xuni(d.ldc);
    P.alpha_re = xunid(d.alpha[0]);
    P.alpha_im = XT<DT>::CPLX ? xunid(d.alpha[1]) : 0.0;
    P.beta_re = xunid(d.beta[0]);
    P.beta_im = XT<DT>::CPLX ? xunid(d.beta[1]) : 0.0;
    const bool a0 = (R)P.alpha_re == (R)0 && (R)P.alpha_im == (R)0;
    const int st = validate(trans, P.m, P.n, P.k, P.lda, P.ldb, P.ldc, a0 ? 0.0f : 1.0f, P.A, P.B, P.C);
    if (status != nullptr && (threadIdx.x & 63) == 0) status[q] = st;
    if (st != 0 || P.m == 0 || P.n == 0) continue;
    if (a0 || P.k == 0) {
      const R br = (R)P.beta_re, bi = (R)P.beta_im;
      for (int64_t e = threadIdx.x & 63; e < (int64_t)P.m * P.n; e += 64) {
        const int64_t ci = e % P.m + (e / P.m) * P.ldc;
        if (br == (R)0 && bi == (R)0) {
          xstore<DT>(P.C, ci, Cx<R>{(R)0, (R)0});
        } else {
          const Cx<R> v = xload<DT>(P.C, ci);
          xstore<DT>(P.C, ci, Cx<R>{br * v.re - bi * v.im, br * v.im + bi * v.re});
        }
      }
      continue;
    }
    switch (trans) {
      case 0: xsolve<DT, 0, 0>(P, table); break;
      case 1: xsolve<DT, 1, 0>(P, table); break;
      case 2: xsolve<DT, 0, 1>(P, table); break;
      default: xsolve<DT, 1, 1>(P, table); break;
    }
  }
}

}  // namespace dev

template <int DT, bool LIGHT>
static void launch_x_kernel(const XProb& P, int layout, int64_t sa, int64_t sb, int64_t sc,
                            int64_t batch, const PlanEntry* table_dev, int nsn, int sb0, int slots,
                            dim3 grid, hipStream_t s) {
  const dim3 block(64);
  switch (layout) {
    case 0: hipLaunchKernelGGL((dev::xgemm_kernel<DT, 0, 0, LIGHT>), grid, block, 0, s, P, sa, sb, sc, batch, table_dev, nsn, sb0, slots); break;
    case 1: hipLaunchKernelGGL((dev::xgemm_kernel<DT, 1, 0, LIGHT>), grid, block, 0, s, P, sa, sb, sc, batch, table_dev, nsn, sb0, slots); break;
    case 2: hipLaunchKernelGGL((dev::xgemm_kernel<DT, 0, 1, LIGHT>), grid, block, 0, s, P, sa, sb, sc, batch, table_dev, nsn, sb0, slots); break;
    default: hipLaunchKernelGGL((dev::xgemm_kernel<DT, 1, 1, LIGHT>), grid, block, 0, s, P, sa, sb, sc, batch, table_dev, nsn, sb0, slots); break;
  }
}

template <int DT>
static hipError_t launch_x_dt(const XProb& P, int layout, int64_t sa, int64_t sb, int64_t sc,
                              int64_t batch, const PlanEntry* table_dev, int nsm, int nsn,
                              int max_blocks, bool light, hipStream_t s) {
  const int64_t es = dev::XT<DT>::CPLX ? 2 * (int64_t)sizeof(typename dev::XT<DT>::R)
                                       : (int64_t)sizeof(typename dev::XT<DT>::R);
  if (max_blocks < 1) return hipSuccess;
  const int64_t nsb = (int64_t)nsm * nsn;
  const int64_t zmax = 0x7fffffffLL / max_blocks;  // grid.x limit
  for (int64_t z0 = 0; z0 < batch; z0 += zmax) {
    const int64_t nz = batch - z0 < zmax ? batch - z0 : zmax;
    XProb Q = P;
    Q.A = (const char*)P.A + es * z0 * sa;
    Q.B = (const char*)P.B + es * z0 * sb;
    Q.C = (char*)P.C + es * z0 * sc;
    for (int64_t s0 = 0; s0 < nsb; s0 += 65535) {  // grid.y limit
      const int64_t ns = nsb - s0 < 65535 ? nsb - s0 : 65535;
      const dim3 grid((unsigned)(nz * max_blocks), (unsigned)ns, 1);
      if (light)
        launch_x_kernel<DT, true>(Q, layout, sa, sb, sc, nz, table_dev, nsn, (int)s0, max_blocks, grid, s);
      else
        launch_x_kernel<DT, false>(Q, layout, sa, sb, sc, nz, table_dev, nsn, (int)s0, max_blocks, grid, s);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_xgemm(int dt, const XProb& P, int layout, int64_t sa, int64_t sb, int64_t sc,
                        int64_t batch, const PlanEntry* table_dev, int nsm, int nsn, int max_blocks,
                        bool light, hipStream_t s) {
  switch (dt) {
    case IAAT_DT_F64: return launch_x_dt<IAAT_DT_F64>(P, layout, sa, sb, sc, batch, table_dev, nsm, nsn, max_blocks, light, s);
    case IAAT_DT_C64: return launch_x_dt<IAAT_DT_C64>(P, layout, sa, sb, sc, batch, table_dev, nsm, nsn, max_blocks, light, s);
    case IAAT_DT_C128: return launch_x_dt<IAAT_DT_C128>(P, layout, sa, sb, sc, batch, table_dev, nsm, nsn, max_blocks, light, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_xscale(int dt, const XProb& P, int64_t sc, int64_t batch, hipStream_t s) {
  const int64_t mn = (int64_t)P.m * P.n;
  const dim3 grid((unsigned)((mn + 255) / 256 < 1024 ? (mn + 255) / 256 : 1024),
                  (unsigned)(batch < 65535 ? batch : 65535)),
      block(256);
  switch (dt) {
    case IAAT_DT_F64: hipLaunchKernelGGL(dev::xscale_kernel<IAAT_DT_F64>, grid, block, 0, s, P, sc, batch); break;
    case IAAT_DT_C64: hipLaunchKernelGGL(dev::xscale_kernel<IAAT_DT_C64>, grid, block, 0, s, P, sc, batch); break;
    case IAAT_DT_C128: hipLaunchKernelGGL(dev::xscale_kernel<IAAT_DT_C128>, grid, block, 0, s, P, sc, batch); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_xgemm_vbatched(int dt, const iaat_xproblem* probs, int64_t count, int32_t* status,
                                 const PlanEntry* table_dev, hipStream_t s) {
  const unsigned grid = (unsigned)(count < (1 << 20) ? count : (1 << 20));
  switch (dt) {
    case IAAT_DT_F64: hipLaunchKernelGGL(dev::xgemm_vbatched_kernel<IAAT_DT_F64>, dim3(grid), dim3(64), 0, s, probs, count, status, table_dev); break;
    case IAAT_DT_C64: hipLaunchKernelGGL(dev::xgemm_vbatched_kernel<IAAT_DT_C64>, dim3(grid), dim3(64), 0, s, probs, count, status, table_dev); break;
    case IAAT_DT_C128: hipLaunchKernelGGL(dev::xgemm_vbatched_kernel<IAAT_DT_C128>, dim3(grid), dim3(64), 0, s, probs, count, status, table_dev); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace iaat
