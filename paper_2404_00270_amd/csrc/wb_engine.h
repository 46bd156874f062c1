// Host engine: many max-flow instances resident in one device arena, solved
// together (their residual graphs form a disjoint union, so one sweep and one
// global relabel serve all of them).  A single solve is an engine holding one
// instance; a batch admits many at once; the server admits new instances
// between rounds while others are still running.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "wb_internal.h"
#include "wb_kernels.h"

namespace wb {

struct SolveConfig {
  int lanes_per_vertex = 0;   // 0: from the mean row length
  int split_degree = 0;       // rows longer than this go to the one-wave tier (0: 4 * lanes)
  int block_degree = 0;       // rows longer than this go to the workgroup tier (0: 2048)
  int gr_every_sweeps = 0;    // fixed sweeps per round (0: adaptive, at most 64)
  int gr_work_permille = 0;   // adaptive relabel budget in thousandths of V + M (0: 1000)
  int64_t max_sweeps = 0;
  int max_wall_ms = 0;
  int grid_blocks = 0;        // workgroups per tile-kernel launch (0: 256)
  bool time_kernels = false;  // bracket every sweep / relabel launch with events
  int push_mode = 0;          // 1: single push to the lowest neighbour; 0/2: full discharge
  bool use_graph = true;      // replay the sweep batch as a captured hipGraph
  bool full_scan = false;     // rebuild the active queue by a full scan every sweep
  int gr_stagnation = 0;      // sweeps without a new smallest queue that end a round (0: by mean row length)
  bool wave_trace = false;    // per-wave execution time and work of every sweep launch
  int lds_max_v = 0;          // instances up to this many vertices are solved in LDS (0: 1024, < 0: never)
  bool gap = true;            // gap heuristic between global relabels (one instance in its phase)
  bool rcsr = false;          // RCSR residual layout (paper section 3.2); else BCSR
  int batch_kernel = 0;       // groups: 0 auto, 1 rounds of launches only, 2 persistent
                              // workgroup-per-instance kernel for every eligible instance
  bool debug_checks = false;  // preflow invariants checked before every global relabel (rounds only)
};

// Counters of the engine since the last reset_stats().
struct EngineStats {
  int lanes = 0, split_degree = 0, block_degree = 0, gr_blocks = 0;
  int64_t sweeps = 0, phase2_sweeps = 0, global_relabels = 0, gr_levels = 0;
  int64_t arc_scans = 0, pushes = 0, relabels = 0, queued = 0, bfs_scans = 0, bfs_topdown_scans = 0;
  int64_t nonempty_sweeps = 0;
  int64_t small_solved = 0;  // instances solved whole in LDS at admission
  int64_t small_fallbacks = 0;  // LDS-resident solves that reached their round cap (rounds finished them)
  int64_t wg_solved = 0;        // instances solved by the persistent workgroup-per-instance kernel
  int64_t wg_fallbacks = 0;     // ... that reached a cap there and were finished by the rounds
  int64_t debug_checked = 0;    // rounds whose state passed the invariant checks (debug_checks)
  int64_t gap_skipped = 0;   // queue entries left to the next global relabel by the gap heuristic
  // per kernel: 0 short-row tiles, 1 medium rows (one wave), 2 long rows (workgroup), 3 global relabel
  double k_ms[4] = {0, 0, 0, 0};
  double build_ms = 0;       // residual-graph builder (event-timed with time_kernels)
  int64_t k_launches[4] = {0, 0, 0, 0};
  int64_t k_scans[4] = {0, 0, 0, 0}, k_pushes[4] = {0, 0, 0, 0}, k_relabels[4] = {0, 0, 0, 0},
          k_queued[4] = {0, 0, 0, 0};
};

// One admission group: n instances whose local CSRs are packed back to back
// in device memory (instance i: V_i + 1 row pointers, E_i columns and
// capacities, local vertex ids).  Outputs are device pointers packed the same
// way (values [n], flows [sum E], sides [sum V]); null = not wanted.
struct GroupInput {
  int32_t n = 0;
  const int32_t *V = nullptr;   // host [n]
  const int64_t *E = nullptr;   // host [n]
  const int32_t *s = nullptr;   // host [n], local ids
  const int32_t *t = nullptr;   // host [n], local ids
  const int64_t *row_ptr = nullptr;  // device, sum(V_i + 1)
  const int32_t *col = nullptr;      // device, sum E_i
  const int32_t *cap = nullptr;      // device, sum E_i
  int64_t *values = nullptr;         // device [n]
  int32_t *flows = nullptr;          // device [sum E]
  uint8_t *sides = nullptr;          // device [sum V]
  uint64_t tag = 0;                  // caller's id, reported back on completion
  bool keep = false;                 // keep the built group after its instances finish (n == 1)
  bool start = true;                 // false: build only, start instances later (start_instance)
  bool persistent = false;           // eligible instances go to the persistent kernel's ring
                                     // (pk_publish) instead of the rounds; nothing is solved here
  int32_t *group_out = nullptr;      // receives the group id (nullable)
};

struct Finished {
  uint64_t tag;     // group tag
  int32_t index;    // instance index inside its group
  int status;       // 0 ok, else a wbpr status code
};

// First-fit allocator of half-open index ranges.
class RangeAlloc {
 public:
  void reset(int64_t cap);
  int64_t alloc(int64_t n);          // -1 when no range fits
  void release(int64_t at, int64_t n);
  void shrink(int64_t at, int64_t n_old, int64_t n_new);
  int64_t largest_free() const;
  int64_t free_total() const { return free_total_; }
  int64_t capacity() const { return cap_; }

 private:
  std::map<int64_t, int64_t> free_;  // start -> length
  int64_t cap_ = 0, free_total_ = 0;
};

class Engine {
 public:
  explicit Engine(int device);
  ~Engine();
  Engine(const Engine &) = delete;
  Engine &operator=(const Engine &) = delete;

  void set_config(const SolveConfig &cfg);
  const SolveConfig &config() const { return cfg_; }

  // Device bytes of an arena for the given capacities (footprint formula).
  static size_t arena_bytes(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap);
  // Device bytes of the per-admission scratch (builder, union CSR staging).
  static size_t scratch_bytes(int64_t V, int64_t E, int32_t n);

  // External memory (the allocation-free entry point): the arena and the
  // builder scratch are carved from [base, base + bytes), which the caller
  // owns and which other users may overwrite between calls, so every
  // reserve() re-carves it for the requested sizes and clears it; host
  // staging is ordinary host memory.  Nothing is allocated on the device and
  // no stream, event or graph is created (sweeps are launched one by one).
  void set_external(void *base, size_t bytes);
  bool external() const { return external_; }
  // Makes room for at least these capacities; only while nothing is
  // resident.  Returns 0 or a wbpr status.
  int reserve(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap, int64_t scratch_V, int64_t scratch_E,
              int32_t scratch_n, std::string *err);
  // Admits a group (builds its residual graphs, preflows them).  Returns 0,
  // WBPR_EAGAIN when the arena has no room now, or another status.
  int admit(const GroupInput &in, hipStream_t st, std::string *err);
  // One round: global relabel of every resident instance, per-instance phase
  // transitions and outputs, then a batch of sweeps.  Appends finished
  // instances to *done.
  int round(hipStream_t st, std::vector<Finished> *done, std::string *err);
  // Starts a new solve on a kept group (built with keep = true): resets its
  // residual capacities from the stored ones (no rebuild), then preflows.
  // s, t are local ids; outputs are device pointers (value required).
  int start_instance(int gid, int32_t s, int32_t t, int64_t *value, int32_t *flow, uint8_t *side, uint64_t tag,
                     hipStream_t st, std::string *err);
  // Releases a kept group that has no running instance.
  void free_group(int gid, hipStream_t st);
  // Runs rounds until nothing is resident.
  int run_to_completion(hipStream_t st, std::vector<Finished> *done, std::string *err);
  // Drops every resident instance (after an error) and clears the arena.
  void abandon(hipStream_t st);

  // Persistent kernel with live admission (the server): instances admitted
  // with GroupInput.persistent are published to a device ring while the
  // kernel runs, and its workgroups claim them; a workgroup exits after
  // kPkIdleMs without an entry.  Never run round() while pk_alive(): the
  // global relabel labels every resident vertex.
  bool pk_alive();
  // (Re)starts the kernel on st_pk when published entries wait and it has exited.
  int pk_ensure_running(hipStream_t st_pk, std::string *err);
  // Reads the results ring (on st, synchronised): finished instances are
  // retired into *done; stopped ones (a cap) join the rounds.
  int pk_collect(hipStream_t st, std::vector<Finished> *done, std::string *err);
  int32_t pk_outstanding() const { return (int32_t)pk_out_.size(); }
  // Instances that need the rounds of launches (too large for the
  // persistent kernel, or stopped at one of its caps).
  int32_t rounds_resident() const;

  bool idle() const { return resident_ == 0; }
  bool has_kept_groups() const;
  int32_t resident() const { return resident_; }
  int64_t free_vertices() const { return valloc_.largest_free(); }
  int64_t free_entries() const { return malloc_.largest_free(); }
  int64_t free_arcs() const { return aalloc_.largest_free(); }
  int32_t free_slots() const { return (int32_t)slot_free_.size(); }
  int64_t last_build_M() const { return last_M_; }
  int64_t sweeps_run() const { return acc_.sweeps; }
  int64_t rounds_run() const { return acc_.global_relabels; }

  void reset_stats();
  // Copies up to cap per-wave trace records of the solve since reset_stats()
  // to host memory; returns the number of records kept (-1 on error).
  int64_t read_wave_trace(hipStream_t st, int32_t *host, int64_t cap, std::string *err);
  int collect_stats(hipStream_t st, EngineStats *out, std::string *err);

 private:
  struct Inst {
    bool used = false;
    int32_t V = 0;
    int64_t E = 0;
    int32_t vbase = 0, s = 0, t = 0;  // arena ids
    int64_t abase = 0;
    int phase = 0;  // 1: max preflow, 2: return excess to s, 3: done, 4: in the persistent kernel
    bool pending_done = false;  // solved whole at admission, retired by the next round
    int32_t maxdeg = 0;  // longest row its sweeps can meet (terminals excluded)
    int group = -1;
    int32_t index = 0;
    int64_t *value = nullptr;
    int32_t *flow = nullptr;
    uint8_t *side = nullptr;
  };
  struct Group {
    bool used = false;
    uint64_t tag = 0;
    int32_t vbase = 0, V = 0;
    int64_t mbase = 0, Mres = 0, abase = 0, E = 0;
    int remaining = 0;
    bool keep = false;
  };

  int ensure_graph(hipStream_t st, int K, int tiers, hipGraphExec_t *exec, std::string *err);
  void carve(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap);
  void reset_books();
  hipError_t ensure_pinned(std::string *err);
  void prime_small_lds();
  int measure_rows(const std::vector<int> &slots, hipStream_t st, std::string *err);
  int solve_small(const std::vector<int> &slots, hipStream_t st, std::string *err);
  int solve_wg(const std::vector<int> &slots, hipStream_t st, std::string *err);
  int debug_check(hipStream_t st, int32_t vhi, std::string *err);
  int pk_publish(const std::vector<int> &slots, hipStream_t st, std::string *err);
  void fill_wg(const struct Inst &I, WgInst *d) const;
  void retire(const std::vector<int> &fin_done, std::vector<Finished> *done, hipStream_t st);
  // persistent kernel state
  WgInst *pk_ring_ = nullptr, *pk_stage_ = nullptr;
  int32_t *pk_result_ = nullptr;
  hipEvent_t pk_ev_ = nullptr;
  bool pk_launched_ = false;
  int32_t pk_tail_ = 0;                          // entries published (host copy)
  std::vector<std::pair<int32_t, int>> pk_out_;  // (entry, instance slot) not yet collected
  int small_lds_ = 0;  // dynamic LDS bytes of the small-instance kernel (0: not yet set, -1: unavailable)
  void drop_graphs();
  void enqueue_sweeps(hipStream_t st, int K, int tiers);
  void launch_inst_kernel(int which, const std::vector<int> &slots, hipStream_t st);
  void launch_inst_list(int which, const std::vector<struct InstDev> &list, const std::vector<int> &slots,
                        hipStream_t st);
  void release_groups(const std::vector<int> &gis, hipStream_t st);
  void dump_sweep_log(hipStream_t st);

  int device_;
  SolveConfig cfg_;
  int gr_blocks_[7] = {0, 0, 0, 0, 0, 0, 0};
  // device memory
  void *arena_ = nullptr;
  size_t arena_n_ = 0;
  void *scratch_ = nullptr;
  size_t scratch_n_ = 0;
  int64_t Vcap_ = 0, Mcap_ = 0, Ecap_ = 0;
  int32_t ncap_ = 0;
  int64_t sV_ = 0, sE_ = 0;
  int32_t sn_ = 0;
  Arena A_;
  long long *e_ = nullptr;
  int32_t *h_ = nullptr, *inst_of_ = nullptr, *q_[2] = {nullptr, nullptr}, *fq_[2] = {nullptr, nullptr};
  int32_t *mid_ = nullptr, *big_ = nullptr, *chunk_w_ = nullptr, *chunk_b_ = nullptr;
  int32_t *task_u_ = nullptr, *task_c_ = nullptr, *lr_cnt_ = nullptr;
  unsigned long long *lr_key_ = nullptr;
  int64_t tcap_ = 0;
  uint8_t *vis_ = nullptr;
  int32_t *gap_hist_ = nullptr;  // gap heuristic: vertices per height above the root
  int64_t nchunk_ = 0;
  int32_t *inst_active_ = nullptr, *inst_stranded_ = nullptr;
  int32_t *roots_ = nullptr, *root_h_ = nullptr, *excl_ = nullptr;
  int2 *dbg_term_ = nullptr;  // debug_checks: {s, t} per instance slot whose vertices are checked ({-1, -1}: none)
  void *inst_list_ = nullptr;  // per-instance kernel descriptors [ncap]
  long long *misc_ = nullptr;
  int32_t *sweep_log_dev_ = nullptr, *sweep_log_ = nullptr;  // log pointer passed to kernels (null: off)
  int32_t *sink_ = nullptr;
  long long *budget_ = nullptr;
  // pinned host staging (external mode: plain host memory)
  char *pin_ = nullptr;
  size_t pin_n_ = 0;
  // external device memory (set_external)
  bool external_ = false;
  void *ext_base_ = nullptr;
  size_t ext_bytes_ = 0;
  std::vector<char> ext_host_;
  // host bookkeeping
  RangeAlloc valloc_, malloc_, aalloc_;
  std::vector<int> slot_free_;
  std::vector<Inst> inst_;
  std::vector<Group> groups_;
  int32_t resident_ = 0;
  int64_t resident_V_ = 0, resident_M_ = 0;
  int64_t last_M_ = 0;
  // what the last round uploaded (roots, their heights, excluded terminals,
  // sink, budget, span): a round that would upload the same skips the copies;
  // emptied when the arena is carved (its memory cleared)
  std::vector<int64_t> gr_uploaded_;
  // tiers and launch shapes (fixed per config)
  int P_ = 8, t_mid_ = 32, t_big_ = 2048, bfs_split_ = 64, chunk_ = BFS_CHUNK, stag_window_ = 16;
  int mid_lanes_ = 64;  // lanes per medium row (16 and 32 measured no faster on R-MAT)
  // captured sweep batches, one per (batch length, tiers); adaptive batch length
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs_;
  int next_K_ = 12, last_K_ = 0;  // multiples of 6
  long long last_nonempty_ = 0;
  // second stream for the long-row chain, which runs beside the medium-row
  // kernel inside a sweep (fork/join events, reused cyclically)
  hipStream_t side_ = nullptr;
  std::vector<hipEvent_t> fork_ev_;
  bool ensure_side();
  // per-wave trace (wave_trace option): int4 records, at most kTraceCap per solve
  static constexpr int32_t kTraceCap = 1 << 22;
  int32_t *wtrace_ = nullptr;
  // timing
  std::vector<hipEvent_t> ev_;
  int ev_used_ = 0;
  std::vector<std::pair<int, int>> ev_marks_;  // (3: relabel, else tiers << 4: sweep; first event)
  EngineStats acc_;
};

}  // namespace wb
