// The request scheduler of the serving loop, independent of HIP: request
// table, admission by memory into a first-fit arena, continuous batching
// into launch slots, completion and latency statistics.  The device work is
// behind an executor (serve.cpp's executor issues the HIP calls; a CPU test
// drives the same scheduler with a fake one):
//
//   bool launch(int slot, const std::vector<Taken>& taken, int64_t n)
//       starts one batched launch of the n GEMMs of `taken` (each request's
//       arena byte offset and GEMMs) on slot `slot`; false if it could not
//       be started (the requests then fail);
//   int query(int slot)      0 still running, 1 done, -1 failed;
//   void drain(int slot)     waits until the slot's work has stopped;
//   void thread_init()       called first on the scheduler thread.
//
// One scheduler thread makes every executor call of a server.  Client
// threads only append requests and read their state; the mutex guards the
// request table, the admission queue and the arena's free list, and is
// released around executor launches.
#pragma once

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/iaat.h"

namespace iaat {
namespace serve {

constexpr int64_t kOutAlign = 64;  // floats: each GEMM's output starts 256-byte aligned

// A GEMM's output footprint in the arena: its C span, ldc*(n-1) + m floats
// (the caller's ldc is kept; the padding after the last column is not).
inline int64_t out_floats(const iaat_problem& p) {
  const int64_t f = (p.m > 0 && p.n > 0) ? (int64_t)p.ldc * (p.n - 1) + p.m : 0;
  return (f + kOutAlign - 1) / kOutAlign * kOutAlign;
}

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

// First-fit allocator over [0, cap) bytes with coalescing frees.
struct Arena {
  std::map<uint64_t, uint64_t> free_blocks;  // byte offset -> size
  uint64_t cap = 0, held = 0, peak_held = 0;

  void reset(uint64_t bytes) {
    cap = bytes;
    free_blocks.clear();
    if (bytes) free_blocks[0] = bytes;
    held = peak_held = 0;
  }

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
};

// One request's part of a launch: its arena byte offset and its GEMMs.
typedef std::pair<uint64_t, std::vector<iaat_problem>> Taken;

struct Slot {
  bool busy = false;
  std::vector<uint64_t> tickets;
};

template <class Exec>
struct Scheduler {
  Exec& exec;
  iaat_serve_cfg cfg{};
  Arena arena;
  std::vector<Slot> slots;
  std::deque<Req> reqs;  // ticket t is reqs[t - 1]
  std::deque<uint64_t> queue;
  int64_t queued_gemms = 0;  // GEMMs of the requests waiting for admission
  int64_t peak_queue = 0;
  int in_flight = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread th;
  bool stopping = false;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  uint64_t launches = 0, done = 0, failed = 0, gemms_done = 0;
  double flops_done = 0, first_arrival = INFINITY, last_done = 0;
  std::vector<double> lat, lag;

  Scheduler(Exec& e, const iaat_serve_cfg& c, int n_slots) : exec(e), cfg(c), slots((size_t)n_slots) {
    arena.reset(c.mem_cap_bytes);
  }

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  void start() {
    t0 = std::chrono::steady_clock::now();
    th = std::thread([this] { run(); });
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
    if (!R.keep) arena.release(R.arena_off, R.bytes);
  }

  void finish_slot(Slot& L, int err, double t) {
    for (uint64_t tk : L.tickets) finish(reqs[tk - 1], err, t);
    L.tickets.clear();
    L.busy = false;
    --in_flight;
  }

  // Completed launches -> done requests.  Caller holds mu.  Every GEMM was
  // validated at submit, so a launch fails only as a whole.
  bool reap() {
    bool any = false;
    for (size_t s = 0; s < slots.size(); ++s) {
      Slot& L = slots[s];
      if (!L.busy) continue;
      const int q = exec.query((int)s);
      if (q == 0) continue;
      finish_slot(L, q > 0 ? 0 : IAAT_ERR_HIP, now());
      any = true;
    }
    if (any) cv_done.notify_all();
    return any;
  }

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

  // Admits queued requests, in arrival order while their outputs fit the
  // arena (the head waits for memory; nothing overtakes it), into free launch
  // slots and launches them.  Caller holds lk; it is released around the
  // executor's launch.
  bool admit(std::unique_lock<std::mutex>& lk) {
    bool any = false;
    for (size_t s = 0; s < slots.size(); ++s) {
      Slot& L = slots[s];
      if (L.busy || !launch_now()) continue;
      int64_t n = 0;
      const double t = now();
      std::vector<Taken> taken;
      while (!queue.empty()) {
        Req& R = reqs[queue.front() - 1];
        if (n > 0 && n + R.n > cfg.max_batch_gemms) break;
        uint64_t off;
        if (!arena.alloc(R.bytes, &off)) break;  // head-of-line waits for memory
        R.arena_off = off;
        R.state = IAAT_REQ_ADMITTED;
        R.t_launch = t;
        L.tickets.push_back(queue.front());
        taken.emplace_back(off, std::move(R.g));
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
      const bool ok = exec.launch((int)s, taken, n);
      lk.lock();
      if (!ok) {  // the requests fail; the slot is reusable once its work has stopped
        exec.drain((int)s);
        finish_slot(L, IAAT_ERR_HIP, now());
        cv_done.notify_all();
      }
    }
    return any;
  }

  void run() {
    exec.thread_init();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      const bool a = reap();
      const bool b = admit(lk);
      if (stopping && queue.empty() && in_flight == 0) break;
      if (a || b) continue;
      if (in_flight > 0 || !queue.empty()) {  // poll completions / the batching window again shortly
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        // an idle wait of at most 1 ms (wait_until on the system clock: the
        // steady-clock form goes through pthread_cond_clockwait, which
        // thread sanitizers of this toolchain do not model)
        cv_work.wait_until(lk, std::chrono::system_clock::now() + std::chrono::milliseconds(1));
      }
    }
  }

  // Appends a request (sizes already checked).  Returns 0, or -1 when the
  // outputs exceed the arena, or -2 when the server is stopping.
  int submit(const iaat_problem* gemms, int64_t count, double t_arrival, bool keep, uint64_t bytes,
             double flops, uint64_t* ticket) {
    if (bytes > cfg.mem_cap_bytes) return -1;
    Req R;
    R.g.assign(gemms, gemms + count);
    R.bytes = bytes;
    R.flops = flops;
    R.n = (int32_t)count;
    R.keep = keep;
    {
      std::lock_guard<std::mutex> lk(mu);
      if (stopping) return -2;
      R.t_submit = now();
      R.t_arrival = t_arrival < 0 ? R.t_submit : t_arrival;
      reqs.push_back(std::move(R));
      *ticket = reqs.size();
      queue.push_back(*ticket);
      queued_gemms += count;
      peak_queue = std::max<int64_t>(peak_queue, (int64_t)queue.size());
    }
    cv_work.notify_one();
    return 0;
  }

  // Frees a kept output: -1 unknown ticket or not kept, -2 not done.
  int release(uint64_t ticket) {
    std::lock_guard<std::mutex> lk(mu);
    if (ticket < 1 || ticket > reqs.size()) return -1;
    Req& R = reqs[ticket - 1];
    if (!R.keep || R.released) return -1;
    if (R.state != IAAT_REQ_DONE) return -2;
    arena.release(R.arena_off, R.bytes);
    R.released = true;
    cv_work.notify_one();
    return 0;
  }

  // Waits until request `ticket` is done.
  void wait(uint64_t ticket) {
    std::unique_lock<std::mutex> lk(mu);
    cv_done.wait(lk, [&] { return reqs[ticket - 1].state == IAAT_REQ_DONE; });
  }

  void stats(iaat_serve_stats* out) {
    std::lock_guard<std::mutex> lk(mu);
    memset(out, 0, sizeof *out);
    out->submitted = reqs.size();
    out->done = done;
    out->failed = failed;
    out->launches = launches;
    out->gemms_done = gemms_done;
    if (!lat.empty()) {
      std::vector<double> v(lat);
      auto q = [&v](double f) {
        const size_t i = std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5));
        std::nth_element(v.begin(), v.begin() + i, v.end());
        return v[i];
      };
      out->p50 = q(0.50);
      out->p99 = q(0.99);
      out->max_latency = *std::max_element(v.begin(), v.end());
      const double span = last_done - first_arrival;
      out->gflops = span > 0 ? flops_done / span / 1e9 : 0.0;
    }
    if (!lag.empty()) {
      std::vector<double> v(lag);
      const size_t i = std::min(v.size() - 1, (size_t)(0.99 * (v.size() - 1) + 0.5));
      std::nth_element(v.begin(), v.begin() + i, v.end());
      out->p99_submit_lag = v[i];
    }
    out->peak_admitted_bytes = arena.peak_held;
    out->peak_queue_depth = peak_queue;
  }

  // Stops accepting requests, lets every queued and running one finish, and
  // joins the scheduler thread.
  void stop() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stopping = true;
    }
    cv_work.notify_all();
    if (th.joinable()) th.join();
  }
};

}  // namespace serve
}  // namespace iaat
