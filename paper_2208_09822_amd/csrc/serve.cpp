// Request loop over the batched form: admission by memory, continuous
// batching into batched launches over several streams, completion by event
// polling, latency statistics, and an open-loop trace replay.
//
// One scheduler thread owns every HIP call of a server.  Client threads only
// append requests (iaat_serve_submit) and read their state; the mutex guards
// the request table, the admission queue and the arena's free list, and is
// released around the HIP calls of a launch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "api_internal.h"
#include "kernels.h"

using namespace iaat;

namespace {

constexpr int64_t kOutAlign = 64;  // floats: each GEMM's output starts 256-byte aligned

struct Req {
  std::vector<iaat_problem> g;  // dropped once launched
  double t_arrival = 0, t_submit = 0, t_launch = -1, t_done = -1;
  uint64_t bytes = 0, arena_off = UINT64_MAX;
  double flops = 0;
  int32_t n = 0;
  int32_t state = IAAT_REQ_QUEUED;
  int32_t err = 0;
  bool keep = false, released = false;
};

// One launch slot.  Its staging buffer holds the launch's descriptors, then
// its output-seeding copy spans, so one upload carries both.
struct Launch {
  char* stage_host = nullptr;  // pinned
  char* stage_dev = nullptr;
  uint32_t* ticket = nullptr;  // window counter of this slot's batched launches (one at a time)
  iaat_problem* desc_host = nullptr;
  CopySpan* cp_host = nullptr;
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  std::vector<int64_t> first;  // first problem of each ticket in the launch
};

// A GEMM's output footprint in the arena: its C span, ldc*(n-1) + m floats
// (the caller's ldc is kept; the padding after the last column is not).
int64_t out_floats(const iaat_problem& p) {
  const int64_t f = (p.m > 0 && p.n > 0) ? (int64_t)p.ldc * (p.n - 1) + p.m : 0;
  return (f + kOutAlign - 1) / kOutAlign * kOutAlign;
}

}  // namespace

struct iaat_server {
  iaat_ctx_t ctx = nullptr;
  iaat_serve_cfg cfg{};
  float* arena = nullptr;
  std::map<uint64_t, uint64_t> free_blocks;  // byte offset -> size
  uint64_t held = 0, peak_held = 0;
  std::vector<hipStream_t> streams;
  std::vector<Launch> slots;
  std::deque<Req> reqs;  // ticket t is reqs[t - 1]
  std::deque<uint64_t> queue;
  int64_t peak_queue = 0;
  int in_flight = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stopping = false;
  std::chrono::steady_clock::time_point t0;
  uint64_t launches = 0, done = 0, failed = 0, gemms_done = 0;
  double flops_done = 0, first_arrival = INFINITY, last_done = 0;
  std::vector<double> lat, lag;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  // First-fit allocation of `bytes` (a multiple of 256) in the arena.
  bool alloc(uint64_t bytes, uint64_t* off) {
    if (bytes == 0) {
      *off = 0;
      return true;
    }
    for (auto it = free_blocks.begin(); it != free_blocks.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const uint64_t rest = it->second - bytes, at = it->first + bytes;
      free_blocks.erase(it);
      if (rest) free_blocks[at] = rest;
      held += bytes;
      peak_held = std::max(peak_held, held);
      return true;
    }
    return false;
  }

  void release(uint64_t off, uint64_t bytes) {
    if (bytes == 0) return;
    held -= bytes;
    auto it = free_blocks.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_blocks.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_blocks.erase(nx);
    }
    if (it != free_blocks.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_blocks.erase(it);
      }
    }
  }

  void finish(Req& R, int err, double t) {
    R.err = err;
    R.state = IAAT_REQ_DONE;
    R.t_done = t;
    ++done;
    if (err) ++failed;
    gemms_done += R.n;
    flops_done += R.flops;
    first_arrival = std::min(first_arrival, R.t_arrival);
    last_done = std::max(last_done, t);
    lat.push_back(t - R.t_arrival);
    lag.push_back(R.t_submit - R.t_arrival);
    if (!R.keep) release(R.arena_off, R.bytes);
  }

  // Completed launches -> done requests.  Caller holds mu.
  bool reap() {
    bool any = false;
    for (Launch& L : slots) {
      if (!L.busy) continue;
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipErrorNotReady) continue;
      const double t = now();
      // every GEMM was validated at submit, so a launch fails only as a whole
      for (size_t r = 0; r < L.tickets.size(); ++r)
        finish(reqs[L.tickets[r] - 1], q == hipSuccess ? 0 : IAAT_ERR_HIP, t);
      L.tickets.clear();
      L.first.clear();
      L.busy = false;
      --in_flight;
      any = true;
    }
    if (any) cv_done.notify_all();
    return any;
  }

  int64_t queued_gemms = 0;  // GEMMs of the requests waiting for admission

  // Continuous batching: with nothing in flight a request is launched at
  // once; while launches are in flight, the next one waits until a quarter
  // of a full launch has queued up or the oldest queued request has waited
  // kBatchWait, so the launch count (and its per-launch host cost) stays
  // bounded under heavy load.
  static constexpr double kBatchWait = 40e-6;
  bool launch_now() const {
    if (queue.empty()) return false;
    if (in_flight == 0 || queued_gemms >= cfg.max_batch_gemms / 4) return true;
    return now() - reqs[queue.front() - 1].t_arrival >= kBatchWait;
  }

  // Admits queued requests into free launch slots and launches them.
  // Caller holds lk; it is released around the HIP calls.
  bool admit(std::unique_lock<std::mutex>& lk) {
    bool any = false;
    for (Launch& L : slots) {
      if (L.busy || !launch_now()) continue;
      int64_t n = 0;
      const double t = now();
      std::vector<std::pair<float*, std::vector<iaat_problem>>> taken;  // output base, GEMMs
      while (!queue.empty()) {
        Req& R = reqs[queue.front() - 1];
        if (n > 0 && n + R.n > cfg.max_batch_gemms) break;
        uint64_t off;
        if (!alloc(R.bytes, &off)) break;  // head-of-line waits for memory
        R.arena_off = off;
        R.state = IAAT_REQ_ADMITTED;
        R.t_launch = t;
        L.tickets.push_back(queue.front());
        L.first.push_back(n);
        taken.emplace_back(arena + off / sizeof(float), std::move(R.g));
        n += R.n;
        queued_gemms -= R.n;
        queue.pop_front();
      }
      if (n == 0) break;  // the head request waits for arena space
      L.busy = true;
      ++in_flight;
      ++launches;
      any = true;
      lk.unlock();
      // outside the lock: descriptors with their outputs in the arena, and
      // the copies that seed outputs from C0 when beta != 0
      int64_t ncp = 0, d = 0;
      for (auto& tk : taken) {
        float* out = tk.first;
        for (const iaat_problem& g : tk.second) {
          iaat_problem p = g;
          p.C = out;
          if (p.beta != 0.0f && p.m > 0 && p.n > 0)
            L.cp_host[ncp++] = CopySpan{g.C, out, (int64_t)p.ldc * (p.n - 1) + p.m};
          L.desc_host[d++] = p;
          out += out_floats(g);
        }
      }
      taken.clear();
      // descriptors then copy spans, contiguous in the slot's staging buffer
      const size_t dbytes = (size_t)n * sizeof(iaat_problem);
      if (ncp > 0) memmove(L.stage_host + dbytes, L.cp_host, (size_t)ncp * sizeof(CopySpan));
      hipError_t e = hipMemcpyAsync(L.stage_dev, L.stage_host, dbytes + (size_t)ncp * sizeof(CopySpan),
                                    hipMemcpyHostToDevice, L.stream);
      if (e == hipSuccess && ncp > 0)
        e = launch_copy_spans((const CopySpan*)(L.stage_dev + dbytes), ncp,
                              (int)std::min<int64_t>(ncp, 4LL * ctx->num_cu), L.stream);
      if (e == hipSuccess)
        e = launch_batch(ctx, (const iaat_problem*)L.stage_dev, n, cfg.prec, nullptr, L.stream,
                         cfg.prec == IAAT_PREC_F32 ? L.ticket : nullptr);
      if (e == hipSuccess) e = hipEventRecord(L.ev, L.stream);
      lk.lock();
      if (e != hipSuccess) {  // the requests fail; the slot is reusable once the stream drains
        (void)hipStreamSynchronize(L.stream);
        for (uint64_t tk : L.tickets) finish(reqs[tk - 1], IAAT_ERR_HIP, now());
        L.tickets.clear();
        L.first.clear();
        L.busy = false;
        --in_flight;
        cv_done.notify_all();
      }
    }
    return any;
  }

  void run() {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      const bool a = reap();
      const bool b = admit(lk);
      if (stopping && queue.empty() && in_flight == 0) break;
      if (a || b) continue;
      if (in_flight > 0 || !queue.empty()) {  // poll the events / batching window again shortly
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv_work.wait_for(lk, std::chrono::milliseconds(1));
      }
    }
  }
};

static void free_server(iaat_server* S) {
  for (Launch& L : S->slots) {
    if (L.stage_host) (void)hipHostFree(L.stage_host);
    if (L.cp_host) (void)hipHostFree(L.cp_host);
    if (L.stage_dev) (void)hipFree(L.stage_dev);
    if (L.ticket) (void)hipFree(L.ticket);
    if (L.ev) (void)hipEventDestroy(L.ev);
  }
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  if (S->arena) (void)hipFree(S->arena);
  delete S;
}

// One tiny GEMM per launch slot on its stream, the way the scheduler
// launches (descriptor upload, a seeding copy, the batched launch with its
// ticket clear), before the server's clock starts: the first use of each
// stream and the first launch of each kernel (code loading) are paid here,
// not by the first requests.  Uses the arena's first 256 bytes (zeros).
static hipError_t warm_slots(iaat_server* S) {
  float* a = S->arena;
  hipError_t e = hipSuccess;
  for (Launch& L : S->slots) {
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
      e = launch_batch(S->ctx, (const iaat_problem*)L.stage_dev, 1, S->cfg.prec, nullptr, L.stream,
                       S->cfg.prec == IAAT_PREC_F32 ? L.ticket : nullptr);
    if (e == hipSuccess) e = hipEventRecord(L.ev, L.stream);
  }
  for (Launch& L : S->slots) {
    const hipError_t q = hipStreamSynchronize(L.stream);
    if (e == hipSuccess) e = q;
  }
  return e;
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
  S->ctx = ctx;
  S->cfg = *cfg;
  const uint64_t cap = cfg->mem_cap_bytes / 256 * 256;
  if (cap == 0 || hipMalloc(&S->arena, cap) != hipSuccess) {
    free_server(S);
    return fail(IAAT_ERR_NOMEM, "iaat_serve_start: arena of %llu bytes", (unsigned long long)cap);
  }
  S->cfg.mem_cap_bytes = cap;
  S->free_blocks[0] = cap;
  const int64_t mb = cfg->max_batch_gemms;
  S->streams.resize(cfg->n_streams, nullptr);
  S->slots.resize(2 * (size_t)cfg->n_streams);
  hipError_t e = hipSuccess;
  for (auto& s : S->streams)
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  for (size_t i = 0; i < S->slots.size() && e == hipSuccess; ++i) {
    Launch& L = S->slots[i];
    L.stream = S->streams[i % S->streams.size()];
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
  if ((e = warm_slots(S)) != hipSuccess) {
    free_server(S);
    return hip_fail(e, "iaat_serve_start: warm-up");
  }
  S->t0 = std::chrono::steady_clock::now();
  S->th = std::thread([S] { S->run(); });
  *out = S;
  return IAAT_OK;
}

// Appends a request; `sizes` (when not NULL) gives the GEMMs' output bytes
// and flops already checked (the replay validates its pool once).
static int submit_request(iaat_server_t S, const iaat_problem* gemms, int64_t count, double t_arrival,
                          int keep_output, uint64_t* ticket, uint64_t bytes, double flops);

int iaat_serve_submit(iaat_server_t S, const iaat_problem* gemms, int64_t count, double t_arrival,
                      int keep_output, uint64_t* ticket) {
  if (!S) return fail(-1, "iaat_serve_submit: server is NULL");
  if (!gemms || count < 1) return fail(-2, "iaat_serve_submit: no GEMMs");
  if (count > S->cfg.max_batch_gemms)
    return fail(-3, "iaat_serve_submit: %lld GEMMs > max_batch_gemms %d", (long long)count,
                S->cfg.max_batch_gemms);
  if (!ticket) return fail(-6, "iaat_serve_submit: ticket is NULL");
  uint64_t bytes = 0;
  double flops = 0;
  for (int64_t i = 0; i < count; ++i) {
    const iaat_problem& p = gemms[i];
    // the output is arena memory; C names the initial value, read only when beta != 0
    static const float dummy = 0.0f;
    int st = validate(p.trans, p.m, p.n, p.k, p.lda, p.ldb, p.ldc, p.alpha, p.A, p.B, &dummy);
    if (st == 0 && p.beta != 0.0f && p.m > 0 && p.n > 0 && p.C == nullptr) st = -13;
    if (st != 0)
      return fail(-4, "iaat_serve_submit: GEMM %lld: argument %d invalid", (long long)i, -st);
    bytes += (uint64_t)out_floats(p) * sizeof(float);
    flops += 2.0 * p.m * (double)p.n * p.k;
  }
  return submit_request(S, gemms, count, t_arrival, keep_output, ticket, bytes, flops);
}

static int submit_request(iaat_server_t S, const iaat_problem* gemms, int64_t count, double t_arrival,
                          int keep_output, uint64_t* ticket, uint64_t bytes, double flops) {
  if (bytes > S->cfg.mem_cap_bytes)
    return fail(-3, "iaat_serve_submit: outputs of %llu bytes exceed the arena",
                (unsigned long long)bytes);
  Req R;
  R.g.assign(gemms, gemms + count);
  R.bytes = bytes;
  R.flops = flops;
  R.n = (int32_t)count;
  R.keep = keep_output != 0;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return fail(IAAT_ERR_UNSUPPORTED, "iaat_serve_submit: server is stopping");
    R.t_submit = S->now();
    R.t_arrival = t_arrival < 0 ? R.t_submit : t_arrival;
    S->reqs.push_back(std::move(R));
    *ticket = S->reqs.size();
    S->queue.push_back(*ticket);
    S->queued_gemms += count;
    S->peak_queue = std::max<int64_t>(S->peak_queue, (int64_t)S->queue.size());
  }
  S->cv_work.notify_one();
  return IAAT_OK;
}

int iaat_serve_poll(iaat_server_t S, uint64_t ticket, iaat_req_status* st) {
  if (!S) return fail(-1, "iaat_serve_poll: server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  if (ticket < 1 || ticket > S->reqs.size()) return fail(-2, "iaat_serve_poll: unknown ticket");
  const Req& R = S->reqs[ticket - 1];
  if (st) {
    st->state = R.state;
    st->err = R.err;
    st->t_arrival = R.t_arrival;
    st->t_launch = R.t_launch;
    st->t_done = R.t_done;
    st->out = (R.keep && !R.released && R.arena_off != UINT64_MAX)
                  ? S->arena + R.arena_off / sizeof(float) : nullptr;
  }
  return R.state == IAAT_REQ_DONE ? 0 : 1;
}

int iaat_serve_release(iaat_server_t S, uint64_t ticket) {
  if (!S) return fail(-1, "iaat_serve_release: server is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  if (ticket < 1 || ticket > S->reqs.size()) return fail(-2, "iaat_serve_release: unknown ticket");
  Req& R = S->reqs[ticket - 1];
  if (!R.keep || R.released) return fail(-2, "iaat_serve_release: output not kept");
  if (R.state != IAAT_REQ_DONE) return fail(-3, "iaat_serve_release: request not done");
  S->release(R.arena_off, R.bytes);
  R.released = true;
  S->cv_work.notify_one();
  return IAAT_OK;
}

double iaat_serve_clock(iaat_server_t S) { return S ? S->now() : 0.0; }

int iaat_serve_stats_get(iaat_server_t S, iaat_serve_stats* out) {
  if (!S) return fail(-1, "iaat_serve_stats_get: server is NULL");
  if (!out) return fail(-2, "iaat_serve_stats_get: out is NULL");
  std::lock_guard<std::mutex> lk(S->mu);
  memset(out, 0, sizeof *out);
  out->submitted = S->reqs.size();
  out->done = S->done;
  out->failed = S->failed;
  out->launches = S->launches;
  out->gemms_done = S->gemms_done;
  if (!S->lat.empty()) {
    std::vector<double> v(S->lat);
    auto q = [&v](double f) {
      const size_t i = std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + i, v.end());
      return v[i];
    };
    out->p50 = q(0.50);
    out->p99 = q(0.99);
    out->max_latency = *std::max_element(v.begin(), v.end());
    const double span = S->last_done - S->first_arrival;
    out->gflops = span > 0 ? S->flops_done / span / 1e9 : 0.0;
  }
  if (!S->lag.empty()) {
    std::vector<double> v(S->lag);
    const size_t i = std::min(v.size() - 1, (size_t)(0.99 * (v.size() - 1) + 0.5));
    std::nth_element(v.begin(), v.begin() + i, v.end());
    out->p99_submit_lag = v[i];
  }
  out->peak_admitted_bytes = S->peak_held;
  out->peak_queue_depth = S->peak_queue;
  return IAAT_OK;
}

int iaat_serve_replay(iaat_server_t S, int64_t n_req, const double* t_arrival,
                      const int32_t* n_gemms, const int64_t* pool_idx, const iaat_problem* pool,
                      int64_t pool_size, double* latency_out) {
  if (!S) return fail(-1, "iaat_serve_replay: server is NULL");
  if (n_req < 0) return fail(-2, "iaat_serve_replay: n_req < 0");
  if (n_req > 0 && (!t_arrival || !n_gemms || !pool_idx || !pool || pool_size < 1))
    return fail(-3, "iaat_serve_replay: missing trace arrays");
  // validate the pool once; per-entry output bytes and flops
  std::vector<uint64_t> pbytes((size_t)pool_size);
  std::vector<double> pflops((size_t)pool_size);
  for (int64_t i = 0; i < pool_size && n_req > 0; ++i) {
    const iaat_problem& p = pool[i];
    static const float dummy = 0.0f;
    int st = validate(p.trans, p.m, p.n, p.k, p.lda, p.ldb, p.ldc, p.alpha, p.A, p.B, &dummy);
    if (st == 0 && p.beta != 0.0f && p.m > 0 && p.n > 0 && p.C == nullptr) st = -13;
    if (st != 0) return fail(-5, "iaat_serve_replay: pool entry %lld: argument %d invalid", (long long)i, -st);
    pbytes[(size_t)i] = (uint64_t)out_floats(p) * sizeof(float);
    pflops[(size_t)i] = 2.0 * p.m * (double)p.n * p.k;
  }
  std::vector<uint64_t> tickets((size_t)n_req, 0);
  std::vector<iaat_problem> g;
  const double t_start = S->now();
  int64_t first = 0;
  int rc = IAAT_OK;
  for (int64_t r = 0; r < n_req && rc == IAAT_OK; ++r) {
    const double target = t_start + t_arrival[r];
    for (double t = S->now(); t < target; t = S->now()) {
      if (target - t > 300e-6)
        std::this_thread::sleep_for(std::chrono::duration<double>(target - t - 200e-6));
      else
        std::this_thread::yield();
    }
    if (n_gemms[r] < 1 || n_gemms[r] > S->cfg.max_batch_gemms) {
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
  std::unique_lock<std::mutex> lk(S->mu);
  for (int64_t r = 0; r < n_req; ++r) {
    if (!tickets[r]) continue;
    S->cv_done.wait(lk, [&] { return S->reqs[tickets[r] - 1].state == IAAT_REQ_DONE; });
    if (latency_out) {
      const Req& R = S->reqs[tickets[r] - 1];
      latency_out[r] = R.t_done - R.t_arrival;
    }
  }
  return rc;
}

int iaat_serve_stop(iaat_server_t S) {
  if (!S) return IAAT_OK;
  {
    DeviceGuard g(S->ctx->device);
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  if (S->th.joinable()) S->th.join();
  DeviceGuard g(S->ctx->device);
  free_server(S);
  return IAAT_OK;
}
