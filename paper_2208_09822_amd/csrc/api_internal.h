// Internals shared by the C ABI sources (api.cpp, serve.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "iaat_internal.h"

struct iaat_vbplan {
  iaat_ctx* ctx = nullptr;
  uint32_t* ticket = nullptr;  // the plan's window counter (cleared at each replay)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t count = 0;
};

struct iaat_hplan {
  iaat_ctx* ctx = nullptr;
  int prec = 0;
  int64_t capacity = 0;
  iaat_problem* host = nullptr;  // pinned staging
  iaat_problem* dev = nullptr;
  uint32_t* ticket = nullptr;    // FP32 window counter
  hipEvent_t done = nullptr;     // the last replay
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int64_t count = -1;            // problems the graph was captured for
};

struct iaat_ctx {
  int device = 0;
  int num_cu = 0;
  int vb_grid = 0;      // batched kernel: work-groups resident at once
  std::vector<iaat::PlanEntry> table;   // the plans in use (host copy of table_dev)
  iaat::PlanEntry* table_dev = nullptr;
  std::vector<iaat::PlanEntry> staged;  // iaat_plan_set edits, applied by iaat_table_commit
  // staging for descriptors handed over in host memory
  std::mutex stage_mu;
  iaat_problem* stage_host = nullptr;
  iaat_problem* stage_dev = nullptr;
  int64_t stage_cap = 0;
  hipEvent_t stage_evt = nullptr;
};

namespace iaat {

// Records the calling thread's error message (iaat_last_error) and returns code.
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Makes `dev` current for the scope, restoring the caller's device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// The batched launch(es) for one device descriptor array.
hipError_t launch_batch(iaat_ctx_t ctx, const iaat_problem* probs_dev, int64_t count, int prec,
                        int32_t* status, hipStream_t s, uint32_t* ticket = nullptr);

}  // namespace iaat
