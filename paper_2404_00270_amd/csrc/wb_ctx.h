// Context object and error plumbing shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <string>

#include "../../include/wbpr.h"
#include "wb_engine.h"

namespace wb {

// Message of the last failing call on this thread (wbpr_last_error).
extern thread_local std::string g_err;

inline int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

inline int hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? WBPR_ENOMEM : WBPR_EDEVICE;
}

// Grow-only device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t n = 0;
  hipError_t ensure(size_t bytes) {
    if (bytes == 0) bytes = 256;
    if (bytes <= n) return hipSuccess;
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    return e;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Host-side validation of one CSR instance (V, E, s, t and, when the arrays
// are host memory, row pointers, columns and capacities).
int check_shape(int32_t V, int64_t E, int32_t s, int32_t t);

}  // namespace wb

struct wbpr_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // order the context stream after a caller's stream (entry) and the
  // caller's stream after the context stream (exit)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  wb::SolveConfig cfg;
  std::unique_ptr<wb::Engine> engine;
  // engine of the allocation-free entry point (carves the static scratch array)
  std::unique_ptr<wb::Engine> engine_na;
  wb::DevBuf input, output;
  // autotuned schedules by shape class (log2 V, log2 mean row length)
  std::map<std::pair<int, int>, wb::SolveConfig> tuned;
};
