// Internal interfaces between the translation units of the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wb {

// ---- primitives (prims.hip)
int64_t scan_temp_elems(int64_t n);
hipError_t excl_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *temp, hipStream_t st);
hipError_t excl_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total, int64_t *temp, hipStream_t st);
int64_t radix_hist_elems(int64_t n);
hipError_t radix_sort_u64_u32(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int bits,
                              int32_t *hist, int32_t *scan_temp, int *result_in_alt, hipStream_t st);

// ---- residual graph: bidirectional CSR with merged entries and explicit
// mate indices (build.hip)
struct Residual {
  int32_t V = 0;
  int64_t E = 0;               // input arcs
  int64_t M = 0;               // merged residual entries (host copy, after build)
  int64_t M_cap = 0;           // capacity of the entry arrays (2E)
  int32_t *rptr = nullptr;     // [V+1] row offsets into ent
  int2 *ent = nullptr;         // [M] {neighbour column, residual capacity}
  int32_t *rev = nullptr;      // [M] index of the mate entry (v,u) of (u,v)
  int32_t *cap0 = nullptr;     // [M] merged forward capacity, sum of c(u->v)
  int32_t *arc2ent = nullptr;  // [E] entry of input arc i, -1 for self-loops
  int32_t *pbefore = nullptr;  // [E] capacity of earlier parallel arcs (u,v)
};

// Status words the builder leaves in device memory.
struct BuildStatus {
  int32_t bad_input;  // validation failures
  int32_t overflow;   // merged pair capacity above INT32_MAX
  int32_t nself;      // self-loops
  int32_t M;          // merged entries
};

// Bytes of the Residual arrays for V vertices and E arcs.
size_t residual_bytes(int32_t V, int64_t E);
// Carves the Residual arrays out of `mem` (residual_bytes() long).
void residual_carve(Residual *res, int32_t V, int64_t E, void *mem);
// Device scratch needed by build_residual.
size_t build_scratch_bytes(int32_t V, int64_t E);

// CSR (device) -> residual graph.  Enqueues everything on `st`; the host
// learns M, validation and overflow results from *status_dev afterwards.
hipError_t build_residual(const int64_t *row_ptr, const int32_t *col, const int32_t *cap, Residual *res,
                          void *scratch, BuildStatus *status_dev, hipStream_t st);

}  // namespace wb
