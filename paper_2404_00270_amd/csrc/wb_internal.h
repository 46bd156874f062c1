// Internal interfaces between the translation units of the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace wb {

// ---- primitives (prims.hip)
int64_t scan_temp_elems(int64_t n);
hipError_t excl_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *temp, hipStream_t st);
int64_t radix_hist_elems(int64_t n);
// passes radix_sort_u64_u32 makes over `bits` key bits (for n > 1); an odd
// count leaves the result in the alternate buffers
int radix_sort_passes(int bits);
// Keys per radix tile and key bits per pass.  hist[d * tiles + b] counts
// the keys of tile b whose digit is d; with first_hist the caller has
// filled it for the first pass (digit bits [shift0, shift0 + RADIX_BITS)).
constexpr int RADIX_TILE = 6144;
constexpr int RADIX_BITS = 8;
hipError_t radix_sort_u64_u32(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int bits,
                              int32_t *hist, int32_t *scan_temp, int *result_in_alt, hipStream_t st, int shift0 = 0,
                              bool first_hist = false);

// ---- residual graph: bidirectional CSR with merged entries and explicit
// mate indices, in a device arena shared by all instances (build.hip)
struct Arena {
  int2 *rowb = nullptr;        // [Vcap] row bounds {first entry, end entry}
  int2 *ent = nullptr;         // [Mcap] {neighbour column, residual capacity}
  int32_t *rev = nullptr;      // [Mcap] BCSR: index of the mate entry (v,u) of (u,v);
                               //        RCSR: flow of the arc at its forward entry
  int32_t *cap0 = nullptr;     // [Mcap] merged forward capacity, sum of c(u->v)
  int32_t *arc2ent = nullptr;  // [Ecap] entry of input arc i, -1 for self-loops
  int32_t *pbefore = nullptr;  // [Ecap] capacity of earlier parallel arcs (u,v)
  int32_t *acap = nullptr;     // [Ecap] input capacity of arc i
};

// Where one build lands in the arena.
struct Place {
  int32_t vbase = 0;  // arena id of local vertex 0
  int64_t mbase = 0;  // first arena entry
  int64_t abase = 0;  // first arena arc slot
};

// Status words the builder leaves in device memory.
struct BuildStatus {
  int32_t bad_input;  // validation failures
  int32_t overflow;   // merged pair capacity above INT32_MAX
  int32_t nself;      // self-loops
  int32_t M;          // merged entries
  int32_t big;        // entries whose summed capacity is at least 2^30 (only
                      // these can overflow int32 together with their mate)
  int32_t unsorted;   // rows whose columns are not non-decreasing
  int32_t nlong;      // groups of equal keys too long for one thread to walk
  int32_t longrun;    // sorted rows holding a run of more than 256 equal columns
};

// Device scratch needed by build_residual for V vertices and E arcs.
size_t build_scratch_bytes(int32_t V, int64_t E);

// CSR (device, local ids 0..V-1) -> residual rows in the arena at `pl`:
// uses at most 2E entries from pl.mbase and E arc slots from pl.abase.
// Enqueues everything on `st`; the host learns M and the validation results
// from *status_dev afterwards.
hipError_t build_residual(const int64_t *row_ptr, const int32_t *col, const int32_t *cap, int32_t V, int64_t E,
                          const Arena &A, const Place &pl, void *scratch, BuildStatus *status_dev, hipStream_t st);

// CSR -> RCSR rows in the arena at `pl` (2E entries: forward then reverse
// entries per row, see build.hip); rev[] of those entries holds the flows.
hipError_t build_residual_rcsr(const int64_t *row_ptr, const int32_t *col, const int32_t *cap, int32_t V, int64_t E,
                               const Arena &A, const Place &pl, void *scratch, BuildStatus *status_dev,
                               hipStream_t st);

}  // namespace wb
