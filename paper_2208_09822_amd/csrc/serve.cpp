// Request loop over the batched form: admission by memory, continuous
// batching into batched launches over several streams, completion by event
// polling, latency statistics, and an open-loop trace replay.
//
// The scheduler itself (request table, arena, batching policy, completion)
// is serve_core.h; this file is its HIP executor -- launch slots with pinned
// staging, streams and events -- and the C ABI.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <thread>
#include <vector>

#include "api_internal.h"
#include "kernels.h"
#include "serve_core.h"

using namespace iaat;
using serve::out_floats;

namespace {

// One launch slot.  Its staging buffer holds the launch's descriptors, then
// its output-seeding copy spans, so one upload carries both.
struct HipSlot {
  char* stage_host = nullptr;  // pinned
  char* stage_dev = nullptr;
  uint32_t* ticket = nullptr;  // window counter of this slot's batched launches (one at a time)
  iaat_problem* desc_host = nullptr;
  CopySpan* cp_host = nullptr;
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
};

struct HipExec {
  iaat_ctx_t ctx = nullptr;
  int prec = IAAT_PREC_F32;
  float* arena = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<HipSlot> slots;

  void thread_init() { (void)hipSetDevice(ctx->device); }

  // Descriptors with their outputs in the arena, the copies that seed
  // outputs from C0 when beta != 0, one upload, the copy kernel and the
  // batched launch, then the slot's completion event.
  bool launch(int s, const std::vector<serve::Taken>& taken, int64_t n) {
    HipSlot& L = slots[(size_t)s];
    int64_t ncp = 0, d = 0;
    for (const serve::Taken& tk : taken) {
      float* out = arena + tk.first / sizeof(float);
      for (const iaat_problem& g : tk.second) {
        iaat_problem p = g;
        p.C = out;
        if (p.beta != 0.0f && p.m > 0 && p.n > 0)
          L.cp_host[ncp++] = CopySpan{g.C, out, (int64_t)p.ldc * (p.n - 1) + p.m};
        L.desc_host[d++] = p;
        out += out_floats(g);
      }
    }
    const size_t dbytes = (size_t)n * sizeof(iaat_problem);
    if (ncp > 0) memmove(L.stage_host + dbytes, L.cp_host, (size_t)ncp * sizeof(CopySpan));
    hipError_t e = hipMemcpyAsync(L.stage_dev, L.stage_host, dbytes + (size_t)ncp * sizeof(CopySpan),
                                  hipMemcpyHostToDevice, L.stream);
    if (e == hipSuccess && ncp > 0)
      e = launch_copy_spans((const CopySpan*)(L.stage_dev + dbytes), ncp,
                            (int)std::min<int64_t>(ncp, 4LL * ctx->num_cu), L.stream);
    if (e == hipSuccess)
      e = launch_batch(ctx, (const iaat_problem*)L.stage_dev, n, prec, nullptr, L.stream,
                       prec == IAAT_PREC_F32 ? L.ticket : nullptr);
    if (e == hipSuccess) e = hipEventRecord(L.ev, L.stream);
    return e == hipSuccess;
  }

  int query(int s) {
    const hipError_t q = hipEventQuery(slots[(size_t)s].ev);
    if (q == hipErrorNotReady) return 0;
    return q == hipSuccess ? 1 : -1;
  }

  void drain(int s) { (void)hipStreamSynchronize(slots[(size_t)s].stream); }

  void free_all() {
    for (HipSlot& L : slots) {
      if (L.stage_host) (void)hipHostFree(L.stage_host);
      if (L.cp_host) (void)hipHostFree(L.cp_host);
      if (L.stage_dev) (void)hipFree(L.stage_dev);
      if (L.ticket) (void)hipFree(L.ticket);
      if (L.ev) (void)hipEventDestroy(L.ev);
    }
    slots.clear();
    for (hipStream_t st : streams) (void)hipStreamDestroy(st);
    streams.clear();
    if (arena) (void)hipFree(arena);
    arena = nullptr;
  }
};

// One tiny GEMM per launch slot on its stream, the way the scheduler
// launches (descriptor upload, a seeding copy, the batched launch with its
// ticket clear), before the server's clock starts: the first use of each
// stream and the first launch of each kernel (code loading) are paid here,
// not by the first requests.  Uses the arena's first 256 bytes (zeros).
hipError_t warm_slots(HipExec& X) {
  float* a = X.arena;
  hipError_t e = hipSuccess;
  for (HipSlot& L : X.slots) {
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, 256, L.stream);
    iaat_problem p{};
    p.A = a;
    p.B = a + 4;
    p.C = a + 8;
    p.m = p.n = p.k = 1;
    p.lda = p.ldb = p.ldc = 1;
    p.alpha = p.beta = p.ab_scale = 1.0f;
    const CopySpan cs{a + 12, a + 8, 1};
    memcpy(L.stage_host, &p, sizeof p);
    memcpy(L.stage_host + sizeof p, &cs, sizeof cs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(L.stage_dev, L.stage_host, sizeof p + sizeof cs, hipMemcpyHostToDevice,
                         L.stream);
    if (e == hipSuccess) e = launch_copy_spans((const CopySpan*)(L.stage_dev + sizeof p), 1, 1, L.stream);
    if (e == hipSuccess)
      e = launch_batch(X.ctx, (const iaat_problem*)L.stage_dev, 1, X.prec, nullptr, L.stream,
                       X.prec == IAAT_PREC_F32 ? L.ticket : nullptr);
    if (e == hipSuccess) e = hipEventRecord(L.ev, L.stream);
  }
  for (HipSlot& L : X.slots) {
    const hipError_t q = hipStreamSynchronize(L.stream);
    if (e == hipSuccess) e = q;
  }
  return e;
}

// Checks one GEMM of a request; its output bytes and flops.  Returns 0 or
// the negative argument number.
int check_gemm(const iaat_problem& p, uint64_t* bytes, double* flops) {
  // the output is arena memory; C names the initial value, read only when beta != 0
  static const float dummy = 0.0f;
  int st = validate(p.trans, p.m, p.n, p.k, p.lda, p.ldb, p.ldc, p.alpha, p.A, p.B, &dummy);
  if (st == 0 && p.beta != 0.0f && p.m > 0 && p.n > 0 && p.C == nullptr) st = -13;
  *bytes = (uint64_t)out_floats(p) * sizeof(float);
  *flops = 2.0 * p.m * (double)p.n * p.k;
  return st;
}

}  // namespace

struct iaat_server {
  HipExec exec;
  serve::Scheduler<HipExec>* core = nullptr;
};

static void free_server(iaat_server* S) {
  delete S->core;
  S->exec.free_all();
  delete S;
}

static int submit_request(iaat_server_t S, const iaat_problem* gemms, int64_t count, double t_arrival,
                          int keep_output, uint64_t* ticket, uint64_t bytes, double flops) {
  const int rc = S->core->submit(gemms, count, t_arrival, keep_output != 0, bytes, flops, ticket);
  if (rc == -1)
    return fail(-3, "iaat_serve_submit: outputs of %llu bytes exceed the arena", (unsigned long long)bytes);
  if (rc == -2) return fail(IAAT_ERR_UNSUPPORTED, "iaat_serve_submit: server is stopping");
  return IAAT_OK;
}

int iaat_serve_start(iaat_ctx_t ctx, const iaat_serve_cfg* cfg, iaat_server_t* out) {
  if (!ctx) return fail(-1, "iaat_serve_start: ctx is NULL");
  if (!cfg || cfg->mem_cap_bytes == 0 || cfg->n_streams < 1 || cfg->n_streams > 16 ||
      cfg->max_batch_gemms < 1 || cfg->prec < IAAT_PREC_F32 || cfg->prec > IAAT_PREC_BF16X3)
    return fail(-2, "iaat_serve_start: bad configuration");
  if (!out) return fail(-3, "iaat_serve_start: out is NULL");
  *out = nullptr;
  DeviceGuard g(ctx->device);
  iaat_server* S = new iaat_server;
  HipExec& X = S->exec;
  X.ctx = ctx;
  X.prec = cfg->prec;
  iaat_serve_cfg c = *cfg;
  c.mem_cap_bytes = cfg->mem_cap_bytes / 256 * 256;
  if (c.mem_cap_bytes == 0 || hipMalloc(&X.arena, c.mem_cap_bytes) != hipSuccess) {
    free_server(S);
    return fail(IAAT_ERR_NOMEM, "iaat_serve_start: arena of %llu bytes",
                (unsigned long long)c.mem_cap_bytes);
  }
  const int64_t mb = cfg->max_batch_gemms;
  X.streams.resize(cfg->n_streams, nullptr);
  X.slots.resize(2 * (size_t)cfg->n_streams);  // two launches in flight per stream
  hipError_t e = hipSuccess;
  for (auto& st : X.streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  for (size_t i = 0; i < X.slots.size() && e == hipSuccess; ++i) {
    HipSlot& L = X.slots[i];
    L.stream = X.streams[i % X.streams.size()];
    const size_t sbytes = mb * (sizeof(iaat_problem) + sizeof(CopySpan));
    if (e == hipSuccess) e = hipHostMalloc((void**)&L.stage_host, sbytes, 0);
    if (e == hipSuccess) e = hipHostMalloc((void**)&L.cp_host, mb * sizeof(CopySpan), 0);
    if (e == hipSuccess) e = hipMalloc((void**)&L.stage_dev, sbytes);
    if (e == hipSuccess) e = hipMalloc((void**)&L.ticket, 256);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&L.ev, hipEventDisableTiming);
    L.desc_host = (iaat_problem*)L.stage_host;
  }
  if (e != hipSuccess) {
    free_server(S);
    return hip_fail(e, "iaat_serve_start: streams and staging");
  }
  if ((e = warm_slots(X)) != hipSuccess) {
    free_server(S);
    return hip_fail(e, "iaat_serve_start: warm-up");
  }
  S->core = new serve::Scheduler<HipExec>(X, c, (int)X.slots.size());
  S->core->start();
  *out = S;
  return IAAT_OK;
}

int iaat_serve_submit(iaat_server_t S, const iaat_problem* gemms, int64_t count, double t_arrival,
                      int keep_output, uint64_t* ticket) {
  if (!S) return fail(-1, "iaat_serve_submit: server is NULL");
  if (!gemms || count < 1) return fail(-2, "iaat_serve_submit: no GEMMs");
  if (count > S->core->cfg.max_batch_gemms)
    return fail(-3, "iaat_serve_submit: %lld GEMMs > max_batch_gemms %d", (long long)count,
                S->core->cfg.max_batch_gemms);
  if (!ticket) return fail(-6, "iaat_serve_submit: ticket is NULL");
  uint64_t bytes = 0;
  double flops = 0;
  for (int64_t i = 0; i < count; ++i) {
    uint64_t b;
    double f;
    const int st = check_gemm(gemms[i], &b, &f);
    if (st != 0)
      return fail(-4, "iaat_serve_submit: GEMM %lld: argument %d invalid", (long long)i, -st);
    bytes += b;
    flops += f;
  }
  return submit_request(S, gemms, count, t_arrival, keep_output, ticket, bytes, flops);
}

int iaat_serve_poll(iaat_server_t S, uint64_t ticket, iaat_req_status* st) {
  if (!S) return fail(-1, "iaat_serve_poll: server is NULL");
  serve::Scheduler<HipExec>& C = *S->core;
  std::lock_guard<std::mutex> lk(C.mu);
  if (ticket < 1 || ticket > C.reqs.size()) return fail(-2, "iaat_serve_poll: unknown ticket");
  const serve::Req& R = C.reqs[ticket - 1];
  if (st) {
    st->state = R.state;
    st->err = R.err;
    st->t_arrival = R.t_arrival;
    st->t_launch = R.t_launch;
    st->t_done = R.t_done;
    st->out = (R.keep && !R.released && R.arena_off != UINT64_MAX)
                  ? S->exec.arena + R.arena_off / sizeof(float) : nullptr;
  }
  return R.state == IAAT_REQ_DONE ? 0 : 1;
}

int iaat_serve_release(iaat_server_t S, uint64_t ticket) {
  if (!S) return fail(-1, "iaat_serve_release: server is NULL");
  const int rc = S->core->release(ticket);
  if (rc == -1) return fail(-2, "iaat_serve_release: unknown ticket or output not kept");
  if (rc == -2) return fail(-3, "iaat_serve_release: request not done");
  return IAAT_OK;
}

double iaat_serve_clock(iaat_server_t S) { return S ? S->core->now() : 0.0; }

int iaat_serve_stats_get(iaat_server_t S, iaat_serve_stats* out) {
  if (!S) return fail(-1, "iaat_serve_stats_get: server is NULL");
  if (!out) return fail(-2, "iaat_serve_stats_get: out is NULL");
  S->core->stats(out);
  return IAAT_OK;
}

int iaat_serve_replay(iaat_server_t S, int64_t n_req, const double* t_arrival,
                      const int32_t* n_gemms, const int64_t* pool_idx, const iaat_problem* pool,
                      int64_t pool_size, double* latency_out) {
  if (!S) return fail(-1, "iaat_serve_replay: server is NULL");
  if (n_req < 0) return fail(-2, "iaat_serve_replay: n_req < 0");
  if (n_req > 0 && (!t_arrival || !n_gemms || !pool_idx || !pool || pool_size < 1))
    return fail(-3, "iaat_serve_replay: missing trace arrays");
  serve::Scheduler<HipExec>& C = *S->core;
  // validate the pool once; per-entry output bytes and flops
  std::vector<uint64_t> pbytes((size_t)pool_size);
  std::vector<double> pflops((size_t)pool_size);
  for (int64_t i = 0; i < pool_size && n_req > 0; ++i) {
    const int st = check_gemm(pool[i], &pbytes[(size_t)i], &pflops[(size_t)i]);
    if (st != 0) return fail(-5, "iaat_serve_replay: pool entry %lld: argument %d invalid", (long long)i, -st);
  }
  std::vector<uint64_t> tickets((size_t)n_req, 0);
  std::vector<iaat_problem> g;
  const double t_start = C.now();
  int64_t first = 0;
  int rc = IAAT_OK;
  for (int64_t r = 0; r < n_req && rc == IAAT_OK; ++r) {
    const double target = t_start + t_arrival[r];
    for (double t = C.now(); t < target; t = C.now()) {
      if (target - t > 300e-6)
        std::this_thread::sleep_for(std::chrono::duration<double>(target - t - 200e-6));
      else
        std::this_thread::yield();
    }
    if (n_gemms[r] < 1 || n_gemms[r] > C.cfg.max_batch_gemms) {
      rc = fail(-4, "iaat_serve_replay: request %lld has %d GEMMs", (long long)r, n_gemms[r]);
      break;
    }
    g.resize((size_t)n_gemms[r]);
    uint64_t bytes = 0;
    double flops = 0;
    for (int32_t i = 0; i < n_gemms[r]; ++i) {
      const int64_t p = pool_idx[first + i];
      if (p < 0 || p >= pool_size) {
        rc = fail(-6, "iaat_serve_replay: pool index %lld", (long long)p);
        break;
      }
      g[i] = pool[p];
      bytes += pbytes[(size_t)p];
      flops += pflops[(size_t)p];
    }
    if (rc != IAAT_OK) break;
    first += n_gemms[r];
    rc = submit_request(S, g.data(), n_gemms[r], target, 0, &tickets[r], bytes, flops);
  }
  // wait for every submitted request
  for (int64_t r = 0; r < n_req; ++r) {
    if (!tickets[r]) continue;
    C.wait(tickets[r]);
    if (latency_out) {
      std::lock_guard<std::mutex> lk(C.mu);
      const serve::Req& R = C.reqs[tickets[r] - 1];
      latency_out[r] = R.t_done - R.t_arrival;
    }
  }
  return rc;
}

int iaat_serve_stop(iaat_server_t S) {
  if (!S) return IAAT_OK;
  DeviceGuard g(S->exec.ctx->device);
  S->core->stop();
  free_server(S);
  return IAAT_OK;
}
