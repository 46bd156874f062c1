// Solver state and driver interface (host side of solve.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "wb_internal.h"

namespace wb {

struct SolveConfig {
  int lanes_per_vertex = 0;   // 0: from the mean row length
  int split_degree = 0;       // rows longer than this go to the one-wave tier (0: 4 * lanes)
  int block_degree = 0;       // rows longer than this go to the workgroup tier (0: 2048)
  int gr_every_sweeps = 0;    // 0: default
  int64_t max_sweeps = 0;
  int max_wall_ms = 0;
  int grid_blocks = 0;        // workgroups per sweep launch (0: default)
  bool time_kernels = false;  // bracket sweep-tile launches with events
  int push_mode = 0;          // 0/2: full discharge, 1: single push to the lowest neighbour
};

// Per-solve device state (vertex arrays, queues, counters).
struct State {
  long long *e = nullptr;     // [V] excess (terminals biased)
  int32_t *h = nullptr;       // [V] height
  int32_t *q[2] = {nullptr, nullptr};   // active-vertex queues
  int32_t *fq[2] = {nullptr, nullptr};  // BFS frontiers
  int32_t *big_v = nullptr;     // long rows of the current sweep
  int32_t *mid_v = nullptr;     // medium rows of the current sweep
  uint8_t *vis = nullptr;       // [V] BFS visit codes
  int32_t *chunk_w = nullptr, *chunk_b = nullptr;
  int64_t nchunk_cap = 0;
  long long *misc = nullptr;  // counters, status, barrier
  static constexpr int kMaxSweeps = 4096;  // sweeps timed per solve
  static constexpr int kMaxGR = 1024;      // global relabels timed per solve
  hipEvent_t (*ev)[4] = nullptr;   // per sweep: before tile, wave, workgroup kernels, after
  hipEvent_t (*gev)[2] = nullptr;  // per global relabel: before, after
  int ev_count = 0, gev_count = 0;
};

struct PhaseStats {
  int64_t sweeps = 0;
  int64_t global_relabels = 0;
  int64_t gr_levels = 0;
};

struct SolveReport {
  int lanes = 0, split_degree = 0, block_degree = 0, gr_blocks = 0;
  // per kernel: 0 short-row tiles, 1 medium rows (one wave), 2 long rows (workgroup), 3 global relabel
  double k_ms[4] = {0, 0, 0, 0};
  int64_t k_launches[4] = {0, 0, 0, 0};
  int64_t k_scans[4] = {0, 0, 0, 0}, k_pushes[4] = {0, 0, 0, 0}, k_relabels[4] = {0, 0, 0, 0},
          k_queued[4] = {0, 0, 0, 0};
  int64_t sweeps = 0, phase2_sweeps = 0, global_relabels = 0;
  int64_t arc_scans = 0, pushes = 0, relabels = 0, queued = 0, bfs_scans = 0, nonempty_sweeps = 0;
  int64_t gr_levels = 0;
  int64_t bfs_topdown_scans = 0;
  double ms_phase1 = 0, ms_phase2 = 0, ms_decode = 0;
};

size_t state_bytes(int32_t V, int64_t Mcap, int chunk);
void state_carve(State *s, int32_t V, int64_t Mcap, int chunk, void *mem);
size_t misc_bytes();
int gr_max_blocks(int device, int lanes);

// Runs both phases on a built residual graph.  Returns 0 or a wbpr status
// code with *err set.  dev_flow / dev_side may be null.
// gr_blocks[i]: co-resident workgroup limit of the global-relabel kernel
// instantiated for 2^i lanes per vertex (i = 2..6).
int solve_on_device(const SolveConfig &cfg, const Residual &res, State &S, int32_t s, int32_t t, const int *gr_blocks,
                    hipStream_t st, long long *pinned, int64_t *dev_value, int32_t *dev_flow, uint8_t *dev_side,
                    const int32_t *dev_cap, SolveReport *rep, std::string *err);

}  // namespace wb
