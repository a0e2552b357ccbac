// The serving scheduler (serve_core.h) behind a fake executor, on the CPU.
// Each check prints "ok <name>" or "FAIL <name>: ..." and the program exits
// with the number of failures.  Built and run by test_serve_scheduler_cpu.py.
#include <stdio.h>

#include <atomic>
#include <chrono>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "serve_core.h"

using iaat::serve::Scheduler;
using iaat::serve::Taken;

static int failures = 0;
#define CHECK(name, cond, ...)                                    \
  do {                                                            \
    if (cond) {                                                   \
      printf("ok %s\n", name);                                    \
    } else {                                                      \
      printf("FAIL %s: ", name);                                  \
      printf(__VA_ARGS__);                                        \
      printf("\n");                                               \
      ++failures;                                                 \
    }                                                             \
  } while (0)

// A launch completes when the test releases it (or at once when `instant`);
// launch number `fail_at` is refused, query of launch `fail_query` reports a
// failure.  Every launch is recorded with its requests' arena offsets.
struct FakeExec {
  std::mutex mu;
  bool instant = true;
  int fail_at = -1, fail_query = -1;
  int n = 0;
  std::vector<int> slot_launch;           // launch number running on each slot
  std::set<int> released;                 // launches allowed to complete
  std::vector<std::vector<uint64_t>> offs;  // per launch: arena offsets in order
  std::vector<int64_t> sizes;             // per launch: GEMM count
  std::vector<int> gemm_m;                // m of every launched GEMM, in launch order
  std::atomic<int> drained{0};

  explicit FakeExec(int slots) : slot_launch((size_t)slots, -1) {}
  void thread_init() {}
  bool launch(int s, const std::vector<Taken>& taken, int64_t count) {
    std::lock_guard<std::mutex> lk(mu);
    const int id = n++;
    std::vector<uint64_t> o;
    for (const Taken& t : taken) {
      o.push_back(t.first);
      for (const iaat_problem& p : t.second) gemm_m.push_back(p.m);
    }
    offs.push_back(o);
    sizes.push_back(count);
    slot_launch[(size_t)s] = id;
    return id != fail_at;
  }
  int query(int s) {
    std::lock_guard<std::mutex> lk(mu);
    const int id = slot_launch[(size_t)s];
    if (!instant && !released.count(id)) return 0;
    return id == fail_query ? -1 : 1;
  }
  void drain(int) { ++drained; }
  int launched() {
    std::lock_guard<std::mutex> lk(mu);
    return n;
  }
  void release_all() {
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < n; ++i) released.insert(i);
  }
};

static iaat_problem gemm(int m, int n) {
  iaat_problem p{};
  p.m = m;
  p.n = n;
  p.k = 4;
  p.lda = m;
  p.ldb = 4;
  p.ldc = m;
  p.alpha = 1.0f;
  p.beta = 0.0f;
  return p;
}

static uint64_t bytes_of(const std::vector<iaat_problem>& g) {
  uint64_t b = 0;
  for (const iaat_problem& p : g) b += (uint64_t)iaat::serve::out_floats(p) * sizeof(float);
  return b;
}

static iaat_serve_cfg cfg_of(uint64_t cap, int max_batch) {
  iaat_serve_cfg c{};
  c.mem_cap_bytes = cap;
  c.n_streams = 1;
  c.max_batch_gemms = max_batch;
  return c;
}

static void wait_all(Scheduler<FakeExec>& S, const std::vector<uint64_t>& tickets) {
  for (uint64_t t : tickets) S.wait(t);
}

int main() {
  // out_floats: the C span ldc*(n-1)+m, rounded up to 64 floats
  {
    iaat_problem p = gemm(10, 3);
    p.ldc = 100;
    CHECK("out_floats_span", iaat::serve::out_floats(p) == 256, "got %lld",
          (long long)iaat::serve::out_floats(p));
    CHECK("out_floats_empty", iaat::serve::out_floats(gemm(0, 5)) == 0, "nonzero");
  }
  // the arena: first fit, coalescing frees, never above the cap
  {
    iaat::serve::Arena A;
    A.reset(4096);
    uint64_t a, b, c, d;
    bool ok = A.alloc(1024, &a) && A.alloc(1024, &b) && A.alloc(1024, &c);
    ok = ok && a == 0 && b == 1024 && c == 2048 && !A.alloc(2048, &d);
    A.release(b, 1024);
    ok = ok && A.alloc(512, &d) && d == 1024;  // first fit reuses the hole
    A.release(d, 512);
    A.release(a, 1024);
    A.release(c, 1024);
    ok = ok && A.free_blocks.size() == 1 && A.free_blocks.begin()->second == 4096 && A.held == 0;
    CHECK("arena_first_fit_coalesce", ok, "free list %zu blocks, held %llu", A.free_blocks.size(),
          (unsigned long long)A.held);
    CHECK("arena_peak", A.peak_held == 3072, "peak %llu", (unsigned long long)A.peak_held);
  }
  // FIFO order, batching cap, admission under a small arena
  {
    FakeExec X(2);
    X.instant = false;
    const uint64_t one = 256;  // bytes of one 1 x 1 output
    Scheduler<FakeExec> S(X, cfg_of(4 * one, 3), 2);
    std::vector<uint64_t> t;
    for (int r = 0; r < 10; ++r) {
      std::vector<iaat_problem> g{gemm(r + 1, 1)};
      uint64_t tk = 0;
      S.submit(g.data(), 1, -1.0, false, bytes_of(g), 1.0, &tk);
      t.push_back(tk);
    }
    S.start();
    // with completions held back, at most 4 outputs (the arena) are admitted
    std::this_thread::sleep_for(std::chrono::milliseconds(50));
    uint64_t held;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      held = S.arena.held;
    }
    CHECK("admission_respects_cap", held <= 4 * one && held > 0, "held %llu", (unsigned long long)held);
    for (int i = 0; i < 200 && X.launched() < 4; ++i) {
      X.release_all();
      std::this_thread::sleep_for(std::chrono::milliseconds(2));
    }
    for (int i = 0; i < 500; ++i) {
      X.release_all();
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
      std::lock_guard<std::mutex> lk(S.mu);
      if (S.done == 10) break;
    }
    wait_all(S, t);
    bool fifo = X.gemm_m.size() == 10;
    for (size_t i = 0; fifo && i < X.gemm_m.size(); ++i) fifo = X.gemm_m[i] == (int)i + 1;
    CHECK("fifo_order", fifo, "launch order differs");
    bool capped = true;
    for (int64_t s : X.sizes) capped = capped && s >= 1 && s <= 3;
    CHECK("batch_cap", capped, "a launch held more than max_batch_gemms");
    iaat_serve_stats st;
    S.stats(&st);
    CHECK("stats_counts", st.done == 10 && st.failed == 0 && st.gemms_done == 10 &&
                              st.peak_admitted_bytes <= 4 * one,
          "done %llu failed %llu peak %llu", (unsigned long long)st.done,
          (unsigned long long)st.failed, (unsigned long long)st.peak_admitted_bytes);
    S.stop();
    CHECK("arena_empty_after", S.arena.held == 0, "held %llu", (unsigned long long)S.arena.held);
  }
  // head-of-line blocking: a request that does not fit yet holds back the
  // ones behind it, even when they would fit
  {
    FakeExec X(2);
    X.instant = false;
    Scheduler<FakeExec> S(X, cfg_of(1024, 8), 2);
    std::vector<uint64_t> t(3);
    std::vector<iaat_problem> big{gemm(1, 1), gemm(1, 1), gemm(1, 1)};  // 768 bytes
    std::vector<iaat_problem> bigger{gemm(1, 1), gemm(1, 1), gemm(1, 1)};
    std::vector<iaat_problem> small{gemm(1, 1)};
    S.submit(big.data(), 3, -1.0, false, bytes_of(big), 3.0, &t[0]);
    S.submit(bigger.data(), 3, -1.0, false, bytes_of(bigger), 3.0, &t[1]);
    S.submit(small.data(), 1, -1.0, false, bytes_of(small), 1.0, &t[2]);
    S.start();
    std::this_thread::sleep_for(std::chrono::milliseconds(30));
    int launched;
    {
      std::lock_guard<std::mutex> lk(X.mu);
      launched = X.n;
    }
    CHECK("head_of_line_waits", launched == 1, "%d launches before the first completed", launched);
    for (int i = 0; i < 500; ++i) {
      X.release_all();
      std::this_thread::sleep_for(std::chrono::milliseconds(1));
      std::lock_guard<std::mutex> lk(S.mu);
      if (S.done == 3) break;
    }
    wait_all(S, t);
    CHECK("head_of_line_order", X.gemm_m.size() == 7, "%zu GEMMs launched", X.gemm_m.size());
    S.stop();
  }
  // a launch that cannot be started fails its requests (the slot is
  // drained) and the server keeps serving; a launch whose completion
  // reports an error fails its requests too
  {
    FakeExec X(2);
    X.fail_at = 0;
    X.fail_query = 1;
    Scheduler<FakeExec> S(X, cfg_of(1 << 20, 1), 2);
    std::vector<uint64_t> t(3);
    for (int r = 0; r < 3; ++r) {
      std::vector<iaat_problem> g{gemm(2, 2)};
      S.submit(g.data(), 1, -1.0, false, bytes_of(g), 8.0, &t[r]);
    }
    S.start();
    wait_all(S, t);
    S.stop();
    std::vector<int> err;
    {
      std::lock_guard<std::mutex> lk(S.mu);
      for (uint64_t tk : t) err.push_back(S.reqs[tk - 1].err);
    }
    CHECK("launch_failure_completes", err[0] == IAAT_ERR_HIP && X.drained == 1,
          "err %d drained %d", err[0], (int)X.drained);
    CHECK("query_failure_completes", err[1] == IAAT_ERR_HIP, "err %d", err[1]);
    CHECK("later_requests_served", err[2] == 0, "err %d", err[2]);
    CHECK("failed_count", S.failed == 2 && S.arena.held == 0, "failed %llu held %llu",
          (unsigned long long)S.failed, (unsigned long long)S.arena.held);
  }
  // stop drains: every request queued before stop completes, and submits
  // after stop are refused
  {
    FakeExec X(4);
    Scheduler<FakeExec> S(X, cfg_of(1 << 20, 4), 4);
    std::vector<uint64_t> t;
    for (int r = 0; r < 50; ++r) {
      std::vector<iaat_problem> g{gemm(1 + r % 5, 2), gemm(3, 3)};
      uint64_t tk = 0;
      S.submit(g.data(), 2, -1.0, r % 7 == 0, bytes_of(g), 1.0, &tk);
      t.push_back(tk);
    }
    S.start();
    S.stop();
    bool all_done = true;
    for (uint64_t tk : t) all_done = all_done && S.reqs[tk - 1].state == IAAT_REQ_DONE;
    CHECK("stop_drains", all_done && S.done == 50, "done %llu", (unsigned long long)S.done);
    std::vector<iaat_problem> g{gemm(1, 1)};
    uint64_t tk = 0;
    CHECK("submit_after_stop", S.submit(g.data(), 1, -1.0, false, 256, 1.0, &tk) == -2, "accepted");
    // kept outputs stay allocated until released
    uint64_t kept_bytes = 0;
    for (uint64_t k : t)
      if (S.reqs[k - 1].keep) kept_bytes += S.reqs[k - 1].bytes;
    CHECK("kept_outputs_held", S.arena.held == kept_bytes, "held %llu kept %llu",
          (unsigned long long)S.arena.held, (unsigned long long)kept_bytes);
    int rel = 0;
    for (uint64_t k : t)
      if (S.reqs[k - 1].keep) rel += S.release(k) == 0;
    CHECK("release_kept", S.arena.held == 0 && rel == 8, "held %llu released %d",
          (unsigned long long)S.arena.held, rel);
    CHECK("release_twice_refused", S.release(t[0]) == -1, "accepted");
  }
  // an oversized request is refused at submit
  {
    FakeExec X(1);
    Scheduler<FakeExec> S(X, cfg_of(512, 4), 1);
    std::vector<iaat_problem> g{gemm(1, 1), gemm(1, 1), gemm(1, 1)};
    uint64_t tk = 0;
    CHECK("oversized_refused", S.submit(g.data(), 3, -1.0, false, bytes_of(g), 1.0, &tk) == -1,
          "accepted");
  }
  return failures;
}
