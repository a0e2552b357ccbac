// C ABI of libiaat (include/iaat.h): context, one-problem calls, batched
// calls, and plan introspection.  Host work per call is O(1); per-problem
// validation and plan lookup of the batched forms run on the device.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "iaat_internal.h"
#include "kernels.h"
#include "tiler.h"
#include "api_internal.h"

using namespace iaat;

namespace {
thread_local std::string g_err;
}  // namespace

namespace iaat {

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(IAAT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace iaat

namespace {

const char* arg_name(int st) {
  switch (st) {
    case -2: return "ta";
    case -3: return "tb/trans";
    case -4: return "m";
    case -5: return "n";
    case -6: return "k";
    case -8: return "A";
    case -9: return "lda";
    case -10: return "B";
    case -11: return "ldb";
    case -13: return "C";
    case -14: return "ldc";
    default: return "?";
  }
}

std::once_flag g_default_checked;
std::string g_default_error;

void free_ctx(iaat_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  if (c->table_dev) (void)hipFree(c->table_dev);
  if (c->stage_dev) (void)hipFree(c->stage_dev);
  if (c->stage_host) (void)hipHostFree(c->stage_host);
  if (c->stage_evt) (void)hipEventDestroy(c->stage_evt);
  delete c;
}

}  // namespace

namespace iaat {

// Blocks of the plan with the most blocks among the (at most four) distinct
// super-block shapes of an m x n problem.
static int max_plan_blocks(iaat_ctx_t ctx, int layout, int64_t m, int64_t n, int64_t nsm, int64_t nsn) {
  const int lm = (int)(m - (nsm - 1) * kSuper), ln = (int)(n - (nsn - 1) * kSuper);
  int maxb = 0;
  const int ms[2] = {kSuper, lm}, ns[2] = {kSuper, ln};
  for (int a = (nsm > 1 ? 0 : 1); a < 2; ++a)
    for (int b = (nsn > 1 ? 0 : 1); b < 2; ++b) {
      const int nb = (int)ctx->table[plan_index(layout, ms[a], ns[b])].nblk;
      if (nb > maxb) maxb = nb;
    }
  return maxb;
}

// Whether every block of the plans a problem uses (its super-blocks' edge
// sizes) is a light family member.
static bool plans_light(iaat_ctx_t ctx, int dt, int layout, int64_t m, int64_t n, int64_t nsm,
                        int64_t nsn) {
  const int lm = (int)(m - (nsm - 1) * kSuper), ln = (int)(n - (nsn - 1) * kSuper);
  const int ms[2] = {kSuper, lm}, ns[2] = {kSuper, ln};
  for (int a = (nsm > 1 ? 0 : 1); a < 2; ++a)
    for (int b = (nsn > 1 ? 0 : 1); b < 2; ++b) {
      const PlanEntry& e = ctx->table[plan_index(layout, ms[a], ns[b])];
      for (uint32_t i = 0; i < e.nblk; ++i)
        if (!kid_is_light(blk_kid(e.blk[i]), dt != IAAT_DT_F64)) return false;
    }
  return true;
}

// The batched launch(es) for one descriptor array: the staged FP32 kernel
// and its companion, or the reduced-precision kernel.
hipError_t launch_batch(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count, int prec,
                        int32_t* status, hipStream_t s, uint32_t* ticket) {
  VbArgs a{probs_dev, count, status, ctx->table_dev, ticket};
  if (prec != IAAT_PREC_F32) {
    // work-groups of four wavefronts, one problem per wavefront (grid-stride)
    const int64_t cap = 8LL * ctx->num_cu, need = (count + 3) / 4;
    return launch_vbatched_lowp(a, prec, (int)(need < cap ? need : cap), s);
  }
  // at most one work-group per 4 problems; each takes windows of up to 16
  // problems (a first one fixed by its index, then claimed from the counter)
  const int64_t units = (count + 3) / 4;
  const int grid = (int)(units < ctx->vb_grid ? units : ctx->vb_grid);
  return launch_vbatched_f32(a, grid, s);
}

}  // namespace iaat

extern "C" {

const char* iaat_last_error(void) { return g_err.c_str(); }

int iaat_create(iaat_ctx_t* out, int device, const char* tile_table_path) {
  g_err.clear();
  if (!out) return fail(-1, "iaat_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(-2, "iaat_create: no HIP device %d (%d visible)", device, ndev);
  DeviceGuard g(device);
  iaat_ctx* c = new iaat_ctx;
  c->device = device;
  std::string why;
  const char* path = tile_table_path;
  if (!path || !*path) path = getenv("IAAT_TILE_TABLE");
  if (path && *path) {
    if (load_table(path, c->table, &why) != 0) {
      delete c;
      return fail(IAAT_ERR_TABLE, "iaat_create: %s", why.c_str());
    }
  } else {
    build_default_table(c->table);
    std::call_once(g_default_checked, [&] {
      for (int lay = 0; lay < kLayouts && g_default_error.empty(); ++lay)
        for (int m = 1; m <= kSuper && g_default_error.empty(); ++m)
          for (int n = 1; n <= kSuper; ++n)
            if (!check_plan(m, n, c->table[plan_index(lay, m, n)], &g_default_error)) break;
    });
    if (!g_default_error.empty()) {
      delete c;
      return fail(IAAT_ERR_TABLE, "iaat_create: built-in table: %s", g_default_error.c_str());
    }
  }
  hipError_t e;
  if ((e = hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, device)) !=
      hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "iaat_create: device attribute");
  }
  int per_cu = 0;
  if ((e = vbatched_occupancy(&per_cu)) != hipSuccess || per_cu < 1) {
    free_ctx(c);
    return hip_fail(e, "iaat_create: occupancy");
  }
  c->vb_grid = per_cu * c->num_cu;
  if ((e = scratch_init(device)) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "iaat_create: scratch address");
  }
  const size_t tbytes = sizeof(PlanEntry) * c->table.size();
  if (hipMalloc(&c->table_dev, tbytes) != hipSuccess) {
    free_ctx(c);
    return fail(IAAT_ERR_NOMEM, "iaat_create: device allocation failed");
  }
  if ((e = hipMemcpy(c->table_dev, c->table.data(), tbytes, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&c->stage_evt, hipEventDisableTiming)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess) {
    free_ctx(c);
    return hip_fail(e, "iaat_create: setup");
  }
  *out = c;
  return IAAT_OK;
}

int iaat_destroy(iaat_ctx_t ctx) {
  free_ctx(ctx);
  return IAAT_OK;
}

int iaat_gemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, float alpha,
              const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
              int64_t ldc, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_gemm: ctx is NULL");
  if (ta != IAAT_OP_N && ta != IAAT_OP_T) return fail(-2, "iaat_gemm: ta=%d", ta);
  if (tb != IAAT_OP_N && tb != IAAT_OP_T) return fail(-3, "iaat_gemm: tb=%d", tb);
  const int layout = ta | (tb << 1);
  const int st = validate(layout, m, n, k, lda, ldb, ldc, alpha, A, B, C);
  if (st != 0)
    return fail(st, "iaat_gemm: invalid %s (m=%lld n=%lld k=%lld lda=%lld ldb=%lld ldc=%lld)",
                arg_name(st), (long long)m, (long long)n, (long long)k, (long long)lda,
                (long long)ldb, (long long)ldc);
  if (m == 0 || n == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (alpha == 0.0f || k == 0) {
    e = launch_scale_f32(C, (int)m, (int)n, (int)ldc, beta, s);
    return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm: scale launch");
  }
  const int64_t nsm = (m + kSuper - 1) / kSuper, nsn = (n + kSuper - 1) / kSuper;
  if (nsm * nsn > 0x7fffffffLL)
    return fail(IAAT_ERR_UNSUPPORTED, "iaat_gemm: %lld x %lld is too large for one launch",
                (long long)m, (long long)n);
  // grid.y = most blocks in any of the (at most four) super-block plans
  const int lm = (int)(m - (nsm - 1) * kSuper), ln = (int)(n - (nsn - 1) * kSuper);
  int maxb = 0;
  const int ms[2] = {kSuper, lm}, ns[2] = {kSuper, ln};
  for (int a = (nsm > 1 ? 0 : 1); a < 2; ++a)
    for (int b = (nsn > 1 ? 0 : 1); b < 2; ++b) {
      const int nb = (int)ctx->table[plan_index(layout, ms[a], ns[b])].nblk;
      if (nb > maxb) maxb = nb;
    }
  dev::Prob P{A, B, C, (int)m, (int)n, (int)k, (int)lda, (int)ldb, (int)ldc, alpha, beta};
  e = launch_gemm_f32(P, layout, ctx->table_dev, (int)nsm, (int)nsn, maxb, s);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm: launch");
}

// Same-size batches the staged batched kernel runs faster than the strided
// kernel (1.2-2x on 40^3, 56^3, 72^3, 80^3, 80x80x16, 48x48x16): both sides
// of C at least 40 and not both multiples of 32, and every operand span
// fits the staging buffer.  Shapes with both sides
// multiples of 32, or one side of 16 or less, stay on the strided kernel,
// whose one-block-per-work-group grid suits them better.
static bool strided_to_staged(int ta, int tb, int64_t m, int64_t n, int64_t k, int64_t lda,
                              int64_t ldb, int64_t ldc) {
  if (m < 40 || n < 40 || m > kSuper || n > kSuper || k > kSuper) return false;
  if (m % 32 == 0 && n % 32 == 0) return false;
  const int64_t sa = ta ? lda * (m - 1) + k : lda * (k - 1) + m;
  const int64_t sb = tb ? ldb * (k - 1) + n : ldb * (n - 1) + k;
  const int64_t sc = ldc * (n - 1) + m;
  return sa + sb + sc <= 19200;  // the largest small-domain problem, 80 x 80 x 80
}

int iaat_gemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                              float alpha, const float* A, int64_t lda, int64_t stride_a,
                              const float* B, int64_t ldb, int64_t stride_b, float beta, float* C,
                              int64_t ldc, int64_t stride_c, int64_t batch, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_gemm_strided_batched: ctx is NULL");
  if (ta != IAAT_OP_N && ta != IAAT_OP_T) return fail(-2, "iaat_gemm_strided_batched: ta=%d", ta);
  if (tb != IAAT_OP_N && tb != IAAT_OP_T) return fail(-3, "iaat_gemm_strided_batched: tb=%d", tb);
  const int layout = ta | (tb << 1);
  int st = validate(layout, m, n, k, lda, ldb, ldc, alpha, A, B, C);
  // argument numbers of this entry point
  static const int remap[15] = {0, 0, -2, -3, -4, -5, -6, 0, -8, -9, -11, -12, 0, -15, -16};
  if (st != 0) {
    st = remap[-st];
    return fail(st, "iaat_gemm_strided_batched: invalid argument %d", -st);
  }
  if (batch < 0) return fail(-18, "iaat_gemm_strided_batched: batch=%lld", (long long)batch);
  if (stride_a < 0) return fail(-10, "iaat_gemm_strided_batched: stride_a=%lld", (long long)stride_a);
  if (stride_b < 0) return fail(-13, "iaat_gemm_strided_batched: stride_b=%lld", (long long)stride_b);
  if (batch > 1 && m > 0 && n > 0 && stride_c < ldc * n)
    return fail(-17, "iaat_gemm_strided_batched: stride_c=%lld < ldc*n (outputs overlap)",
                (long long)stride_c);
  if (m == 0 || n == 0 || batch == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (alpha == 0.0f || k == 0) {
    e = launch_scale_f32_strided(C, (int)m, (int)n, (int)ldc, beta, stride_c, batch, s);
    return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_strided_batched: scale launch");
  }
  const int64_t nsm = (m + kSuper - 1) / kSuper, nsn = (n + kSuper - 1) / kSuper;
  if (nsm * nsn > 0x7fffffffLL)
    return fail(IAAT_ERR_UNSUPPORTED, "iaat_gemm_strided_batched: %lld x %lld is too large",
                (long long)m, (long long)n);
  dev::Prob P{A, B, C, (int)m, (int)n, (int)k, (int)lda, (int)ldb, (int)ldc, alpha, beta};
  if (batch <= 0x7fffffffLL && strided_to_staged(ta, tb, m, n, k, lda, ldb, ldc)) {
    // the staged batched kernel, on descriptors written on the device (the
    // same blocks in the same order: bitwise the same C)
    iaat_problem* d = nullptr;
    e = hipMallocAsync((void**)&d, (size_t)batch * sizeof(iaat_problem), s);
    if (e == hipSuccess) {
      e = launch_strided_desc(d, batch, P, layout, stride_a, stride_b, stride_c, s);
      if (e == hipSuccess) e = launch_batch(ctx, d, batch, IAAT_PREC_F32, nullptr, s);
      const hipError_t ef = hipFreeAsync(d, s);
      if (e == hipSuccess) e = ef;
      return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_strided_batched: staged launch");
    }
    (void)hipGetLastError();  // no stream-ordered memory: the strided kernel below
  }
  e = launch_gemm_f32_strided(P, layout, ctx->table_dev, (int)nsm, (int)nsn,
                              max_plan_blocks(ctx, layout, m, n, nsm, nsn), stride_a, stride_b,
                              stride_c, batch, s);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_strided_batched: launch");
}

// DGEMM / CGEMM / ZGEMM, one problem or a same-size strided batch: the
// FP32 path's argument checks, then the plan-driven family kernels.
static int x_strided(iaat_ctx_t ctx, int dt, const char* name, int ta, int tb, int64_t m, int64_t n,
                     int64_t k, double alpha_re, double alpha_im, const void* A, int64_t lda,
                     int64_t stride_a, const void* B, int64_t ldb, int64_t stride_b, double beta_re,
                     double beta_im, void* C, int64_t ldc, int64_t stride_c, int64_t batch,
                     iaat_stream_t stream) {
  if (!ctx) return fail(-1, "%s: ctx is NULL", name);
  if (ta != IAAT_OP_N && ta != IAAT_OP_T) return fail(-2, "%s: ta=%d", name, ta);
  if (tb != IAAT_OP_N && tb != IAAT_OP_T) return fail(-3, "%s: tb=%d", name, tb);
  const int layout = ta | (tb << 1);
  const bool a0 = alpha_re == 0.0 && alpha_im == 0.0;
  // validate reads alpha only as "is it zero"
  int st = validate(layout, m, n, k, lda, ldb, ldc, a0 ? 0.0f : 1.0f, A, B, C);
  static const int remap[15] = {0, 0, -2, -3, -4, -5, -6, 0, -8, -9, -11, -12, 0, -15, -16};
  if (st != 0) {
    st = remap[-st];
    return fail(st, "%s: invalid argument %d", name, -st);
  }
  if (batch < 0) return fail(-18, "%s: batch=%lld", name, (long long)batch);
  if (stride_a < 0) return fail(-10, "%s: stride_a=%lld", name, (long long)stride_a);
  if (stride_b < 0) return fail(-13, "%s: stride_b=%lld", name, (long long)stride_b);
  if (batch > 1 && m > 0 && n > 0 && stride_c < ldc * n)
    return fail(-17, "%s: stride_c=%lld < ldc*n (outputs overlap)", name, (long long)stride_c);
  if (m == 0 || n == 0 || batch == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  XProb P{A, B, C, (int)m, (int)n, (int)k, (int)lda, (int)ldb, (int)ldc,
          alpha_re, alpha_im, beta_re, beta_im};
  hipError_t e;
  if (a0 || k == 0) {
    e = launch_xscale(dt, P, stride_c, batch, s);
  } else {
    const int64_t nsm = (m + kSuper - 1) / kSuper, nsn = (n + kSuper - 1) / kSuper;
    if (nsm * nsn > 0x7fffffffLL)
      return fail(IAAT_ERR_UNSUPPORTED, "%s: %lld x %lld is too large", name, (long long)m,
                  (long long)n);
    e = launch_xgemm(dt, P, layout, stride_a, stride_b, stride_c, batch, ctx->table_dev, (int)nsm,
                     (int)nsn, max_plan_blocks(ctx, layout, m, n, nsm, nsn),
                     plans_light(ctx, dt, layout, m, n, nsm, nsn), s);
  }
  return e == hipSuccess ? IAAT_OK : hip_fail(e, name);
}

// Argument numbers of the one-problem signatures, from the strided ones.
static int one_problem_rc(int rc) {
  static const int back[19] = {0, -1, -2, -3, -4, -5, -6, -7, -8, -9, 0, -10, -11, 0, -12, -13, -14, 0, 0};
  return (rc < 0 && rc > -19) ? back[-rc] : rc;
}

int iaat_dgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               double alpha, const double* A, int64_t lda, int64_t stride_a,
                               const double* B, int64_t ldb, int64_t stride_b, double beta,
                               double* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream) {
  return x_strided(ctx, IAAT_DT_F64, "iaat_dgemm", ta, tb, m, n, k, alpha, 0.0, A, lda, stride_a, B,
                   ldb, stride_b, beta, 0.0, C, ldc, stride_c, batch, stream);
}

int iaat_dgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
               int64_t ldc, iaat_stream_t stream) {
  return one_problem_rc(iaat_dgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, 0, B, ldb, 0,
                                                   beta, C, ldc, 0, 1, stream));
}

int iaat_cgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               const float* alpha, const void* A, int64_t lda, int64_t stride_a,
                               const void* B, int64_t ldb, int64_t stride_b, const float* beta,
                               void* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_cgemm: ctx is NULL");
  if (!alpha) return fail(-7, "iaat_cgemm: alpha is NULL");
  if (!beta) return fail(-14, "iaat_cgemm: beta is NULL");
  return x_strided(ctx, IAAT_DT_C64, "iaat_cgemm", ta, tb, m, n, k, alpha[0], alpha[1], A, lda,
                   stride_a, B, ldb, stride_b, beta[0], beta[1], C, ldc, stride_c, batch, stream);
}

int iaat_cgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, const float* alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, const float* beta, void* C,
               int64_t ldc, iaat_stream_t stream) {
  return one_problem_rc(iaat_cgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, 0, B, ldb, 0,
                                                   beta, C, ldc, 0, 1, stream));
}

int iaat_zgemm_strided_batched(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k,
                               const double* alpha, const void* A, int64_t lda, int64_t stride_a,
                               const void* B, int64_t ldb, int64_t stride_b, const double* beta,
                               void* C, int64_t ldc, int64_t stride_c, int64_t batch,
                               iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_zgemm: ctx is NULL");
  if (!alpha) return fail(-7, "iaat_zgemm: alpha is NULL");
  if (!beta) return fail(-14, "iaat_zgemm: beta is NULL");
  return x_strided(ctx, IAAT_DT_C128, "iaat_zgemm", ta, tb, m, n, k, alpha[0], alpha[1], A, lda,
                   stride_a, B, ldb, stride_b, beta[0], beta[1], C, ldc, stride_c, batch, stream);
}

int iaat_zgemm(iaat_ctx_t ctx, int ta, int tb, int64_t m, int64_t n, int64_t k, const double* alpha,
               const void* A, int64_t lda, const void* B, int64_t ldb, const double* beta, void* C,
               int64_t ldc, iaat_stream_t stream) {
  return one_problem_rc(iaat_zgemm_strided_batched(ctx, ta, tb, m, n, k, alpha, A, lda, 0, B, ldb, 0,
                                                   beta, C, ldc, 0, 1, stream));
}

int iaat_xgemm_vbatched(iaat_ctx_t ctx, int dtype, const iaat_xproblem* probs_dev, int64_t count,
                        int32_t* status_dev, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_xgemm_vbatched: ctx is NULL");
  if (count < 0 || count > (1LL << 40))
    return fail(-3, "iaat_xgemm_vbatched: count=%lld", (long long)count);
  if (count > 0 && !probs_dev) return fail(-2, "iaat_xgemm_vbatched: probs is NULL");
  if (dtype != IAAT_DT_F64 && dtype != IAAT_DT_C64 && dtype != IAAT_DT_C128)
    return fail(-4, "iaat_xgemm_vbatched: dtype=%d", dtype);
  if (count == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_xgemm_vbatched(dtype, probs_dev, count, status_dev, ctx->table_dev,
                                             (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_xgemm_vbatched: launch");
}

struct iaat_tradplan {
  iaat_ctx* ctx = nullptr;
  TradProb* probs = nullptr;
  int32_t* tiles = nullptr;
  float* work = nullptr;
  int64_t count = 0, ntiles = 0, work_floats = 0;
};

int iaat_trad_destroy(iaat_tradplan_t p) {
  if (!p) return IAAT_OK;
  DeviceGuard g(p->ctx->device);
  if (p->probs) (void)hipFree(p->probs);
  if (p->tiles) (void)hipFree(p->tiles);
  if (p->work) (void)hipFree(p->work);
  delete p;
  return IAAT_OK;
}

int iaat_trad_create(iaat_ctx_t ctx, const iaat_problem* probs_host, int64_t count,
                     iaat_tradplan_t* out) {
  if (!ctx) return fail(-1, "iaat_trad_create: ctx is NULL");
  if (count < 0 || (count > 0 && !probs_host)) return fail(-2, "iaat_trad_create: no problems");
  if (!out) return fail(-4, "iaat_trad_create: out is NULL");
  *out = nullptr;
  std::vector<TradProb> tp((size_t)count);
  std::vector<int32_t> tiles;
  int64_t work = 0;
  for (int64_t q = 0; q < count; ++q) {
    const iaat_problem& d = probs_host[q];
    const int st = validate(d.trans, d.m, d.n, d.k, d.lda, d.ldb, d.ldc, d.alpha, d.A, d.B, d.C);
    if (st != 0) return fail(-2, "iaat_trad_create: problem %lld: argument %d invalid", (long long)q, -st);
    if (d.m > 0x3fffffff / 16 || q > 0x7fffffff)
      return fail(IAAT_ERR_UNSUPPORTED, "iaat_trad_create: problem %lld too large", (long long)q);
    TradProb& P = tp[(size_t)q];
    P.A = (const float*)d.A;
    P.B = (const float*)d.B;
    P.C = d.C;
    P.m = d.m; P.n = d.n; P.k = d.k;
    P.lda = d.lda; P.ldb = d.ldb; P.ldc = d.ldc;
    P.trans = d.trans;
    P.alpha = d.alpha * d.ab_scale;
    P.beta = d.beta;
    P.m16 = (d.m + 15) / 16 * 16;
    P.n16 = (d.n + 15) / 16 * 16;
    P.k16 = (P.alpha == 0.0f) ? 0 : (d.k + 15) / 16 * 16;
    P.a_off = work;
    work += ((int64_t)P.m16 * P.k16 + 63) / 64 * 64;
    P.b_off = work;
    work += ((int64_t)P.n16 * P.k16 + 63) / 64 * 64;
    for (int ti = 0; ti < P.m16 / 16; ++ti)
      for (int tj = 0; tj < P.n16 / 16; ++tj) {
        tiles.push_back((int32_t)q);
        tiles.push_back(ti);
        tiles.push_back(tj);
      }
  }
  DeviceGuard g(ctx->device);
  iaat_tradplan* p = new iaat_tradplan;
  p->ctx = ctx;
  p->count = count;
  p->ntiles = (int64_t)tiles.size() / 3;
  p->work_floats = work;
  hipError_t e = hipSuccess;
  if (count > 0) e = hipMalloc(&p->probs, tp.size() * sizeof(TradProb));
  if (e == hipSuccess && p->ntiles > 0) e = hipMalloc(&p->tiles, tiles.size() * sizeof(int32_t));
  if (e == hipSuccess && work > 0) e = hipMalloc(&p->work, work * sizeof(float));
  if (e == hipSuccess && count > 0)
    e = hipMemcpy(p->probs, tp.data(), tp.size() * sizeof(TradProb), hipMemcpyHostToDevice);
  if (e == hipSuccess && p->ntiles > 0)
    e = hipMemcpy(p->tiles, tiles.data(), tiles.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    iaat_trad_destroy(p);
    return fail(IAAT_ERR_NOMEM, "iaat_trad_create: workspace of %lld floats: %s", (long long)work,
                hipGetErrorString(e));
  }
  *out = p;
  return IAAT_OK;
}

int64_t iaat_trad_workspace_bytes(iaat_tradplan_t p) { return p ? p->work_floats * 4 : 0; }

int iaat_trad_pack(iaat_tradplan_t p, iaat_stream_t stream) {
  if (!p) return fail(-1, "iaat_trad_pack: plan is NULL");
  if (p->count == 0 || p->work_floats == 0) return IAAT_OK;
  DeviceGuard g(p->ctx->device);
  const int64_t cap = 8LL * p->ctx->num_cu;
  const hipError_t e = launch_trad_pack(p->probs, p->count, p->work,
                                        (int)(p->count < cap ? p->count : cap), (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_trad_pack: launch");
}

int iaat_trad_compute(iaat_tradplan_t p, iaat_stream_t stream) {
  if (!p) return fail(-1, "iaat_trad_compute: plan is NULL");
  if (p->ntiles == 0) return IAAT_OK;
  DeviceGuard g(p->ctx->device);
  const int64_t cap = 64LL * p->ctx->num_cu;
  const hipError_t e = launch_trad_tiles(p->probs, p->tiles, p->ntiles, p->work,
                                         (int)(p->ntiles < cap ? p->ntiles : cap), (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_trad_compute: launch");
}

int iaat_quantize_batch(iaat_ctx_t ctx, int prec, const iaat_qjob* jobs_dev, int64_t count,
                        iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_quantize_batch: ctx is NULL");
  if (prec < IAAT_PREC_BF16 || prec > IAAT_PREC_BF16X3)
    return fail(-2, "iaat_quantize_batch: prec=%d is not a reduced-precision mode", prec);
  if (count < 0) return fail(-4, "iaat_quantize_batch: count=%lld", (long long)count);
  if (count > 0 && !jobs_dev) return fail(-3, "iaat_quantize_batch: jobs is NULL");
  if (count == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  const int64_t cap = 8LL * ctx->num_cu;
  const hipError_t e = launch_quantize(prec, jobs_dev, count, (int)(count < cap ? count : cap),
                                       (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_quantize_batch: launch");
}

int iaat_gemm_vbatched_device(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count,
                              int prec, int32_t* status, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_gemm_vbatched_device: ctx is NULL");
  if (count < 0 || count > 0x7fffffffLL)
    return fail(-3, "iaat_gemm_vbatched_device: count=%lld", (long long)count);
  if (count > 0 && !probs_dev) return fail(-2, "iaat_gemm_vbatched_device: probs is NULL");
  if (prec < IAAT_PREC_F32 || prec > IAAT_PREC_BF16X3) return fail(-4, "iaat_gemm_vbatched_device: prec=%d", prec);
  if (count == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  hipStream_t s = (hipStream_t)stream;
  const hipError_t e = launch_batch(ctx, probs_dev, count, prec, status, s);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_vbatched_device: launch");
}

// Largest batch of the allocation-free form: the window counter in the
// device scratch is 32 bits wide.
constexpr int64_t kNoAllocMaxCount = 0x7fffffffLL;

int iaat_gemm_vbatched_noalloc(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count,
                               int32_t* status, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_gemm_vbatched_noalloc: ctx is NULL");
  if (count < 0 || count > kNoAllocMaxCount)
    return fail(-3, "iaat_gemm_vbatched_noalloc: count=%lld outside [0, %lld] (the scratch "
                "window counter is 32 bits)", (long long)count, (long long)kNoAllocMaxCount);
  if (count > 0 && !probs_dev) return fail(-2, "iaat_gemm_vbatched_noalloc: probs is NULL");
  if (count == 0) return IAAT_OK;
  uint32_t* ticket = scratch_address(ctx->device);
  if (!ticket) return fail(IAAT_ERR_HIP, "iaat_gemm_vbatched_noalloc: no scratch on device %d",
                           ctx->device);
  DeviceGuard g(ctx->device);
  const hipError_t e = launch_batch(ctx, probs_dev, count, IAAT_PREC_F32, status,
                                    (hipStream_t)stream, ticket);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_vbatched_noalloc: launch");
}

int iaat_vbplan_create(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count, int prec,
                       int32_t* status, iaat_vbplan_t* out) {
  if (!ctx) return fail(-1, "iaat_vbplan_create: ctx is NULL");
  if (count < 0 || count > 0x7fffffffLL)
    return fail(-3, "iaat_vbplan_create: count=%lld", (long long)count);
  if (count > 0 && !probs_dev) return fail(-2, "iaat_vbplan_create: probs is NULL");
  if (prec < IAAT_PREC_F32 || prec > IAAT_PREC_BF16X3) return fail(-4, "iaat_vbplan_create: prec=%d", prec);
  if (!out) return fail(-6, "iaat_vbplan_create: out is NULL");
  *out = nullptr;
  DeviceGuard g(ctx->device);
  iaat_vbplan* p = new iaat_vbplan;
  p->ctx = ctx;
  p->count = count;
  hipStream_t cs = nullptr;
  hipError_t e;
  auto cleanup = [&](int rc) {
    if (cs) (void)hipStreamDestroy(cs);
    if (p->ticket) (void)hipFree(p->ticket);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
    return rc;
  };
  // FP32 replays hand windows out dynamically from the plan's own counter
  if (prec == IAAT_PREC_F32 && (e = hipMalloc((void**)&p->ticket, 256)) != hipSuccess)
    return cleanup(fail(IAAT_ERR_NOMEM, "iaat_vbplan_create: ticket counter"));
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return cleanup(hip_fail(e, "iaat_vbplan_create: capture setup"));
  if (count > 0) {
    e = launch_batch(ctx, probs_dev, count, prec, status, cs, p->ticket);
    if (e != hipSuccess) {
      hipGraph_t tmp = nullptr;
      (void)hipStreamEndCapture(cs, &tmp);
      if (tmp) (void)hipGraphDestroy(tmp);
      return cleanup(hip_fail(e, "iaat_vbplan_create: captured launch"));
    }
  }
  if ((e = hipStreamEndCapture(cs, &p->graph)) != hipSuccess ||
      (e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0)) != hipSuccess ||
      (e = hipDeviceSynchronize()) != hipSuccess)
    return cleanup(hip_fail(e, "iaat_vbplan_create: instantiate"));
  (void)hipStreamDestroy(cs);
  *out = p;
  return IAAT_OK;
}

int iaat_vbplan_launch(iaat_vbplan_t plan, iaat_stream_t stream) {
  if (!plan) return fail(-1, "iaat_vbplan_launch: plan is NULL");
  DeviceGuard g(plan->ctx->device);
  const hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_vbplan_launch");
}

int iaat_vbplan_destroy(iaat_vbplan_t plan) {
  if (!plan) return IAAT_OK;
  DeviceGuard g(plan->ctx->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->ticket) (void)hipFree(plan->ticket);
  delete plan;
  return IAAT_OK;
}

int iaat_vbatched_plan(iaat_ctx_t ctx, int64_t capacity, int prec, iaat_hplan_t* out) {
  if (!ctx) return fail(-1, "iaat_vbatched_plan: ctx is NULL");
  if (capacity < 1 || capacity > 0x7fffffffLL)
    return fail(-2, "iaat_vbatched_plan: capacity=%lld", (long long)capacity);
  if (prec < IAAT_PREC_F32 || prec > IAAT_PREC_BF16X3) return fail(-3, "iaat_vbatched_plan: prec=%d", prec);
  if (!out) return fail(-4, "iaat_vbatched_plan: out is NULL");
  *out = nullptr;
  DeviceGuard g(ctx->device);
  iaat_hplan* p = new iaat_hplan;
  p->ctx = ctx;
  p->prec = prec;
  p->capacity = capacity;
  const size_t bytes = (size_t)capacity * sizeof(iaat_problem);
  hipError_t e = hipHostMalloc((void**)&p->host, bytes, 0);
  if (e == hipSuccess) e = hipMalloc((void**)&p->dev, bytes);
  if (e == hipSuccess && prec == IAAT_PREC_F32) e = hipMalloc((void**)&p->ticket, 256);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    iaat_vbatched_free(p);
    return fail(IAAT_ERR_NOMEM, "iaat_vbatched_plan: %lld descriptors", (long long)capacity);
  }
  *out = p;
  return IAAT_OK;
}

// Captures the descriptor upload and the batched launch for `count` problems.
static hipError_t hplan_capture(iaat_hplan* p, int64_t count) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  p->count = -1;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    if (cs) (void)hipStreamDestroy(cs);
    return e;
  }
  hipError_t le = hipSuccess;
  if (count > 0) {
    le = hipMemcpyAsync(p->dev, p->host, (size_t)count * sizeof(iaat_problem), hipMemcpyHostToDevice, cs);
    if (le == hipSuccess) le = launch_batch(p->ctx, p->dev, count, p->prec, nullptr, cs, p->ticket);
  }
  e = hipStreamEndCapture(cs, &p->graph);
  (void)hipStreamDestroy(cs);
  if (le != hipSuccess) return le;
  if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
  if (e == hipSuccess) p->count = count;
  return e;
}

int iaat_vbatched_run(iaat_hplan_t p, const iaat_problem* probs_host, int64_t count,
                      iaat_stream_t stream) {
  if (!p) return fail(-1, "iaat_vbatched_run: plan is NULL");
  if (count < 0 || count > p->capacity)
    return fail(-3, "iaat_vbatched_run: count=%lld outside [0, %lld]", (long long)count,
                (long long)p->capacity);
  if (count > 0 && !probs_host) return fail(-2, "iaat_vbatched_run: probs is NULL");
  DeviceGuard g(p->ctx->device);
  // the previous replay's upload has read the staging once this event is done
  hipError_t e = hipEventSynchronize(p->done);
  if (e != hipSuccess) return hip_fail(e, "iaat_vbatched_run: wait");
  if (count > 0) memcpy(p->host, probs_host, (size_t)count * sizeof(iaat_problem));
  if (count != p->count && (e = hplan_capture(p, count)) != hipSuccess)
    return hip_fail(e, "iaat_vbatched_run: capture");
  e = hipGraphLaunch(p->exec, (hipStream_t)stream);
  if (e == hipSuccess) e = hipEventRecord(p->done, (hipStream_t)stream);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_vbatched_run: launch");
}

int iaat_vbatched_free(iaat_hplan_t p) {
  if (!p) return IAAT_OK;
  DeviceGuard g(p->ctx->device);
  if (p->done) (void)hipEventSynchronize(p->done);
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->ticket) (void)hipFree(p->ticket);
  if (p->dev) (void)hipFree(p->dev);
  if (p->host) (void)hipHostFree(p->host);
  if (p->done) (void)hipEventDestroy(p->done);
  delete p;
  return IAAT_OK;
}

int iaat_gemm_vbatched(iaat_ctx_t ctx, const iaat_problem* probs_host, int64_t count, int prec,
                       int32_t* status, iaat_stream_t stream) {
  if (!ctx) return fail(-1, "iaat_gemm_vbatched: ctx is NULL");
  if (count < 0 || count > 0x7fffffffLL)
    return fail(-3, "iaat_gemm_vbatched: count=%lld", (long long)count);
  if (count > 0 && !probs_host) return fail(-2, "iaat_gemm_vbatched: probs is NULL");
  if (prec < IAAT_PREC_F32 || prec > IAAT_PREC_BF16X3) return fail(-4, "iaat_gemm_vbatched: prec=%d", prec);
  if (count == 0) return IAAT_OK;
  DeviceGuard g(ctx->device);
  std::lock_guard<std::mutex> lk(ctx->stage_mu);
  hipError_t e = hipEventSynchronize(ctx->stage_evt);  // previous staged batch consumed
  if (e != hipSuccess) return hip_fail(e, "iaat_gemm_vbatched: staging wait");
  if (count > ctx->stage_cap) {
    if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
    if (ctx->stage_dev) (void)hipFree(ctx->stage_dev);
    ctx->stage_host = nullptr;
    ctx->stage_dev = nullptr;
    ctx->stage_cap = 0;
    const int64_t cap = count < 1024 ? 1024 : count;
    if (hipHostMalloc(&ctx->stage_host, cap * sizeof(iaat_problem)) != hipSuccess ||
        hipMalloc(&ctx->stage_dev, cap * sizeof(iaat_problem)) != hipSuccess)
      return fail(IAAT_ERR_NOMEM, "iaat_gemm_vbatched: staging allocation of %lld failed",
                  (long long)cap);
    ctx->stage_cap = cap;
  }
  hipStream_t s = (hipStream_t)stream;
  memcpy(ctx->stage_host, probs_host, count * sizeof(iaat_problem));
  e = hipMemcpyAsync(ctx->stage_dev, ctx->stage_host, count * sizeof(iaat_problem),
                     hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "iaat_gemm_vbatched: descriptor upload");
  const int rc = iaat_gemm_vbatched_device(ctx, ctx->stage_dev, count, prec, status, stream);
  if (rc != IAAT_OK) return rc;
  e = hipEventRecord(ctx->stage_evt, s);
  return e == hipSuccess ? IAAT_OK : hip_fail(e, "iaat_gemm_vbatched: event");
}

static int describe_plan(const PlanEntry& e, int m, int n, iaat_block* out, int cap) {
  for (uint32_t b = 0; b < e.nblk && (int)b < cap; ++b) {
    const int i0 = blk_i0(e.blk[b]), j0 = blk_j0(e.blk[b]), kid = blk_kid(e.blk[b]);
    const KidInfo& k = kKids[kid];
    out[b].i0 = i0;
    out[b].j0 = j0;
    out[b].rows = (i0 + k.rows < m ? i0 + k.rows : m) - i0;
    out[b].cols = (j0 + k.cols < n ? j0 + k.cols : n) - j0;
    out[b].kid = kid;
  }
  return (int)e.nblk;
}

int iaat_plan_query(iaat_ctx_t ctx, int layout, int m, int n, iaat_block* out, int cap) {
  if (!ctx) return fail(-1, "iaat_plan_query: ctx is NULL");
  if (layout < 0 || layout > 3) return fail(-2, "iaat_plan_query: layout=%d", layout);
  if (m < 1 || m > kSuper) return fail(-3, "iaat_plan_query: m=%d", m);
  if (n < 1 || n > kSuper) return fail(-4, "iaat_plan_query: n=%d", n);
  if (cap < 0 || (cap > 0 && !out)) return fail(-6, "iaat_plan_query: cap=%d", cap);
  return describe_plan(ctx->table[plan_index(layout, m, n)], m, n, out, cap);
}

int iaat_default_plan(int layout, int m, int n, iaat_block* out, int cap) {
  if (layout < 0 || layout > 3) return fail(-1, "iaat_default_plan: layout=%d", layout);
  if (m < 1 || m > kSuper) return fail(-2, "iaat_default_plan: m=%d", m);
  if (n < 1 || n > kSuper) return fail(-3, "iaat_default_plan: n=%d", n);
  if (cap < 0 || (cap > 0 && !out)) return fail(-5, "iaat_default_plan: cap=%d", cap);
  return describe_plan(default_plan(layout, m, n), m, n, out, cap);
}

int iaat_plan_set(iaat_ctx_t ctx, int layout, int m, int n, const iaat_block* blocks, int nblk) {
  if (!ctx) return fail(-1, "iaat_plan_set: ctx is NULL");
  if (layout < 0 || layout > 3) return fail(-2, "iaat_plan_set: layout=%d", layout);
  if (m < 1 || m > kSuper) return fail(-3, "iaat_plan_set: m=%d", m);
  if (n < 1 || n > kSuper) return fail(-4, "iaat_plan_set: n=%d", n);
  if (!blocks) return fail(-5, "iaat_plan_set: blocks is NULL");
  if (nblk < 1 || nblk > kMaxBlocks) return fail(-6, "iaat_plan_set: nblk=%d", nblk);
  PlanEntry e;
  memset(&e, 0, sizeof e);
  e.nblk = (uint32_t)nblk;
  for (int b = 0; b < nblk; ++b) {
    const iaat_block& x = blocks[b];
    if (x.kid < 0 || x.kid >= IAAT_NUM_KIDS || x.i0 < 0 || x.i0 >= m || x.j0 < 0 || x.j0 >= n)
      return fail(-5, "iaat_plan_set: block %d (kid %d at %d,%d)", b, x.kid, x.i0, x.j0);
    e.blk[b] = pack_block(x.i0, x.j0, x.kid);
  }
  std::string why;
  if (!check_plan(m, n, e, &why)) return fail(-5, "iaat_plan_set: %s", why.c_str());
  if (ctx->staged.empty()) ctx->staged = ctx->table;
  ctx->staged[plan_index(layout, m, n)] = e;
  return IAAT_OK;
}

int iaat_table_commit(iaat_ctx_t ctx) {
  if (!ctx) return fail(-1, "iaat_table_commit: ctx is NULL");
  if (ctx->staged.empty()) return IAAT_OK;
  DeviceGuard g(ctx->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(ctx->table_dev, ctx->staged.data(), ctx->staged.size() * sizeof(PlanEntry),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "iaat_table_commit: upload");
  ctx->table.swap(ctx->staged);
  ctx->staged.clear();

  return IAAT_OK;
}

int iaat_table_save(iaat_ctx_t ctx, const char* path) {
  if (!ctx) return fail(-1, "iaat_table_save: ctx is NULL");
  if (!path || !*path) return fail(-2, "iaat_table_save: path is empty");
  std::string why;
  const int rc = save_table(path, ctx->table, &why);
  return rc == 0 ? IAAT_OK : fail(rc, "%s", why.c_str());
}

int iaat_family_size(void) { return IAAT_NUM_KIDS; }

int iaat_family_dtypes(int32_t* codes, int cap) {
  static const int32_t kCodes[IAAT_NUM_DTYPES] = {
#define IAAT_DT_CODE(code, letter) code,
      IAAT_FOR_EACH_DTYPE(IAAT_DT_CODE)
#undef IAAT_DT_CODE
  };
  if (codes)
    for (int i = 0; i < IAAT_NUM_DTYPES && i < cap; ++i) codes[i] = kCodes[i];
  return IAAT_NUM_DTYPES;
}

int iaat_staged_unit_count(void) { return IAAT_NUM_STAGED_UNITS; }

int iaat_staged_unit_info(int unit, int32_t* family, int32_t* p1, int32_t* p2) {
  static const int32_t kUnits[IAAT_NUM_STAGED_UNITS][3] = {
#define IAAT_UNIT_INFO(uid, fam, a, b) {fam, a, b},
      IAAT_FOR_EACH_STAGED_UNIT(IAAT_UNIT_INFO)
#undef IAAT_UNIT_INFO
  };
  if (unit < 0 || unit >= IAAT_NUM_STAGED_UNITS) return fail(-1, "iaat_staged_unit_info: unit=%d", unit);
  if (family) *family = kUnits[unit][0];
  if (p1) *p1 = kUnits[unit][1];
  if (p2) *p2 = kUnits[unit][2];
  return IAAT_OK;
}

int iaat_family_info(int kid, int32_t* family, int32_t* p1, int32_t* p2, int32_t* block_rows,
                     int32_t* block_cols) {
  if (kid < 0 || kid >= IAAT_NUM_KIDS) return fail(-1, "iaat_family_info: kid=%d", kid);
  const KidInfo& k = kKids[kid];
  if (family) *family = k.fam;
  if (p1) *p1 = k.p1;
  if (p2) *p2 = k.p2;
  if (block_rows) *block_rows = k.rows;
  if (block_cols) *block_cols = k.cols;
  return IAAT_OK;
}

int iaat_in_small_domain(int layout, int64_t m, int64_t n, int64_t k) {
  if (layout < 0 || layout > 3) return fail(-1, "iaat_in_small_domain: layout=%d", layout);
  if (m < 0) return fail(-2, "iaat_in_small_domain: m < 0");
  if (n < 0) return fail(-3, "iaat_in_small_domain: n < 0");
  if (k < 0) return fail(-4, "iaat_in_small_domain: k < 0");
  return in_small_domain(layout, m, n, k) ? 1 : 0;
}

}  // extern "C"
