// Kernel argument blocks and launch wrappers of the sweep and global-relabel
// kernels (solve.hip), shared with the host engine (engine.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wb_common.h"

namespace wb {

constexpr int SWEEP_THREADS = 256;
constexpr int BLK = 256;
constexpr int GR_THREADS = 1024;
// Height cap: a vertex of instance i has height hcap - V_i + (local height);
// local height >= V_i, i.e. h >= hcap, means inactive; hcap + 1 marks the
// terminal a phase never labels.
constexpr int32_t HCAP = 1 << 30;
// Long rows are cut into tasks of CHUNK entries, one workgroup each.
constexpr int32_t CHUNK = 1024;
// Gap heuristic: heights counted above the root (a gap among them cuts off
// every vertex above it, counted or not).
constexpr int32_t GAP_BINS = 256;
// The relabel's bottom-up pass cuts rows longer than its split degree into
// BFS_CHUNK-entry pieces, one wave each.
constexpr int32_t BFS_CHUNK = 1024;

// Residual layouts (paper, section 3.2), the template flag RC of every
// kernel that reads rows:
//   BCSR (RC false): one entry per ordered vertex pair, {column, residual},
//     rows sorted by column; the mate (v,u) of entry (u,v) is rev[k].
//   RCSR (RC true): row u lists the arcs leaving u as forward entries
//     {column, residual} (read coalesced), then the arcs entering u as
//     reverse entries {column | RC_REV, index of the arc's forward entry}.
//     The residual of a reverse entry is the arc's flow, flow[index]: one
//     gather per entry, the cost the paper weighs against BCSR's search for
//     the mate.  A push along forward entry k moves d from ent[k].y to
//     flow[k]; along a reverse entry with index j, from flow[j] to ent[j].y.
// A push handle names the two words a push moves capacity between: the
// entry position k (BCSR, RCSR forward) or ~j (RCSR reverse).
constexpr int32_t RC_REV = (int32_t)0x80000000;

template <bool RC>
__device__ __forceinline__ int32_t col_of(int2 cr) {
  return RC ? (cr.x & 0x7fffffff) : cr.x;
}

template <bool RC>
__device__ __forceinline__ int32_t handle_of(int32_t k, int2 cr) {
  return RC && cr.x < 0 ? ~cr.y : k;
}

// Residual capacity of an entry whose words are cr (plain loads: a stale
// value only delays a push or relabel to a later visit).
template <bool RC>
__device__ __forceinline__ int32_t res_of(const int32_t *flow, int2 cr) {
  return RC && cr.x < 0 ? flow[cr.y] : cr.y;
}

// Residual capacity of the mate of entry k: the arc from the entry's
// column back into the row's vertex (the global relabel's top-down step).
template <bool RC>
__device__ __forceinline__ int32_t mate_res(const int2 *ent, const int32_t *rev, const int32_t *flow, int32_t k,
                                            int2 cr) {
  if (!RC) return ent[rev[k]].y;
  return cr.x < 0 ? ent[cr.y].y : flow[k];
}

struct Graph {
  int32_t V;             // arena vertices
  int32_t hcap;          // height cap: h >= hcap is inactive
  const int2 *rowb;      // row bounds {first entry, end entry}
  int2 *ent;
  const int32_t *rev;    // BCSR: mate of every entry
  int32_t *flow;         // RCSR: flow of every arc, at its forward entry
  long long *e;
  int32_t *h;
  const int32_t *sink;   // target whose excess is never read, so pushes into
                         // it skip the excess atomic (-1: none skipped)
  // Gap heuristic (nullable; written by the global relabel): gap[0] lowest
  // height found empty since the relabel (hcap: none), gap[1] the root's
  // height, gap[2] the heights counted (<= GAP_BINS; 0: heuristic off);
  // gap_hist[d] the vertices at height gap[1] + d.
  int32_t *gap_hist;
  int32_t *gap;
};

struct SweepQ {
  const int32_t *qin;
  const int32_t *qin_cnt;
  int32_t *qout;
  int32_t *qout_cnt;
  int32_t *zero_cnt;
  int32_t *mid_v;       // medium rows deferred to the one-wave tier
  int32_t *mid_cnt;
  int32_t *big_v;       // long rows deferred to the chunk kernel (first chunk)
  int32_t *big_cnt;
  int32_t *task_u;      // further chunks of long rows: vertex ...
  int32_t *task_c;      // ... and chunk index within its row
  int32_t *task_cnt;
  int32_t tcap;         // capacity of the task arrays (V + M / CHUNK + 64)
  int32_t *zero_c;      // task counter to clear for the next sweep
  unsigned long long *lr_key;     // per vertex: minimum (height, position) key over its chunks
  int32_t *lr_cnt;                // per vertex: CHUNK_MORE when a chunk left admissible capacity unpushed
  int32_t *zero_a;      // counters to clear for the next sweep (nullable)
  int32_t *zero_b;
  int32_t t_mid;        // rows longer than this go to the one-wave tier
  int32_t t_big;        // rows longer than this go to the workgroup tier
  long long *stats;     // per kernel k (0 tile, 1 wave, 2 workgroup): [4k] arc scans, [4k+1] pushes,
                        // [4k+2] relabels, [4k+3] queued; [12] bfs scans; [13] nonempty sweeps
  long long *rwork;     // running sum of row lengths scanned by relabels
  // nullable: per-workgroup partial counters, PART_SLOTS slots of PART_WORDS
  // (one cache line each: [0..11] as stats[0..11], [12] relabel work, [13]
  // gap skips as stats[15]), which
  // the control step folds into stats and rwork; without it the kernels add
  // to stats and rwork directly
  long long *part;
  int32_t sofs;         // this launch's offset into stats ([4k] of its kernel k above)
  const int32_t *halt;  // set by k_sweep_control: the rest of this round's sweeps do nothing
  int32_t qcap;      // capacity of every queue and of the medium-row list (V)
  int32_t *err;      // overflow counter (must stay 0)
  int32_t mode;      // 0: one push to the minimum-height neighbour (Algorithms 1-2)
                     // 1: full discharge (push along every lower residual arc, then relabel)
  int32_t append;    // 1: append push targets and still-active vertices to qout (incremental
                     // queue); 0: the next sweep's full scan finds them
  int32_t *wtrace;   // nullable: per-wave records (int4: sweep * 4 + kind, ticks, scans, items)
  int32_t *wtrace_n; // records written so far (may exceed wtrace_cap: the excess is dropped)
  int32_t wtrace_cap;
  const int32_t *sweep_no;  // sweeps completed since the solve started (counted by the control step)
  int32_t kind;      // 0 short-row tiles, 1 medium rows, 2 first chunks, 3 further chunks
  long long *gap_skips;  // queue entries left to the next global relabel by the gap heuristic
};

constexpr int PART_SLOTS = 64;  // = the control step's threads (one wave)
constexpr int PART_WORDS = 16;

// End-of-sweep control (one thread after the fold): halt decision and optional log.
struct SweepCtl {
  const int32_t *qin_cnt, *mid_cnt, *big_cnt, *task_cnt, *qout_cnt;
  const long long *rwork, *rwork_at_gr, *budget;
  int32_t *halt;
  int32_t *scan_cnt; // nullable: full-scan queue count, cleared here for the next scan
  int32_t *stag;     // [2] smallest queue of this round, sweeps since it was reached (reset by the relabel)
  int32_t stag_window;  // sweeps without a new smallest queue that end the round
  int32_t *log;      // nullable: [log_cap][6] per-sweep records
  int32_t *log_n;
  int32_t log_cap;
  int32_t *sweep_no;  // nullable: incremented once per sweep that ran
  long long *part;    // nullable: per-workgroup partial counters to fold ...
  long long *stats;   // ... into these counters [0..11] ...
  long long *rwork_acc;  // ... and into the relabel work (the rwork above)
};

struct GRArgs {
  Graph g;
  const int32_t *roots;    // [nroots] BFS sources (the phase's target of every instance)
  const int32_t *root_h;   // [nroots] their heights (per-instance base hcap - V_i)
  int32_t nroots;
  const int32_t *excl;     // [nexcl] terminals that are never labelled
  int32_t nexcl;
  const int32_t *inst_of;  // [V] instance slot of every arena vertex (-1: free)
  int32_t *inst_active;    // per instance: active vertices after this relabel
  int32_t *inst_stranded;  // per instance: excess vertices that cannot reach the root
  int32_t ninst;           // instance slots (inst_active and inst_stranded are cleared first)
  int32_t *fq[2];
  int32_t *fcnt;      // [3] rotating frontier counters
  uint8_t *vis;       // [V] 0 unvisited, 1/2 labelled at even/odd distance, 3 excluded
  int32_t *chunk_w;   // long rows: vertex
  int32_t *chunk_b;   //            first entry of the chunk
  int32_t *chunk_cnt; // [2]
  int32_t *bucnt;     // [3] rotating counts of vertices labelled by bottom-up steps
  long long *fedges;  // [3] rotating row-length sums of the next frontier
  unsigned *bar;      // barrier state (WB_BAR_WORDS)
  int32_t *qout;      // active-vertex queue rebuilt at the end
  int32_t *qcnt;      // [3] sweep counters: [0] = queue length, [1],[2] zeroed
  int32_t *big_cnt;   // [2] zeroed
  int32_t *mid_cnt;   // [2] zeroed
  int32_t *task_cnt;  // [2] zeroed
  long long *stats;
  long long *status;  // [0] active, [1] stranded, [2] levels, [3] bottom-up levels
  int32_t split_deg, chunk;
  int32_t qcap;       // capacity of frontiers and queue (V)
  int32_t chunk_cap;  // capacity of the chunk descriptor arrays
  int32_t bu_threshold;    // frontier size above which a level runs bottom-up
  long long bu_edges;      // frontier row-length sum above which a level runs bottom-up
  long long m_total;       // entries of all resident rows (unvisited edges = m_total - visited)
  int32_t *err;       // overflow counter (must stay 0)
  int32_t *halt;          // sweep halt flag, cleared here
  const long long *rwork; // relabel work so far ...
  long long *rwork_at_gr; // ... snapshot at this global relabel
  int32_t *stag;          // [2] stagnation state of the sweeps, reset here
  uint32_t *bm;           // 4 bitmaps of bm_words words: visited, then three rotating frontiers
  int32_t bm_words;       // words per bitmap (>= V / 32)
  long long *tlog;        // nullable (diagnostics): per level {wall clock, frontier, bottom-up}
  int32_t tlog_cap;
  int32_t gap_base;       // gap heuristic (g.gap non-null): the one root's height ...
  int32_t gap_n;          // ... and heights counted from it (<= GAP_BINS; 0: off this round)
};

// Persistent batched solve (wgsolve.hip): one workgroup of WG_THREADS per
// instance, instances claimed from a work queue in list order.
constexpr int WG_THREADS = 256;

struct WgInst {
  int32_t vbase, V, s, t;  // arena ids of local vertex 0, s and t
  int64_t abase, E;        // input-arc range (flow decode)
  long long *value;        // outputs (device, nullable but value)
  int32_t *flow;
  uint8_t *side;
  int32_t lanes;           // tile width of the sweeps: 1, 4, 8, 16, 32 or 64
  int32_t budget_pm;       // relabel work between BFSs, thousandths of V + M (0: 1000)
};

struct WgArgs {
  const WgInst *L;
  int32_t n;               // list entries
  int32_t *head;           // claim counter (0 at launch)
  const int32_t *tail;     // nullable: entries published so far (persistent mode); else all n
  const int32_t *close;    // nullable (persistent mode): nonzero once nothing more will be published
  long long idle_ticks;    // persistent mode: a workgroup exits after this long without an entry
  int32_t ring;            // persistent mode: entry i lives in slot i % ring of L and result (0: no ring)
  int32_t *result;         // per entry: 1 solved, 2 stopped in phase 1, 3 stopped in phase 2
  const int2 *rowb;
  int2 *ent;
  int32_t *rev;            // BCSR mates / RCSR flows
  const int32_t *cap0;
  const int32_t *arc2ent;
  const int32_t *pbefore;
  const int32_t *acap;
  long long *e;
  int32_t *h;
  int32_t *qa, *qb;        // vertex lists: an instance uses its vertex range of each
  long long *stats;        // nullable: scans, pushes, relabels, sweeps, BFS rounds, BFS scans
  int32_t round_cap;       // BFS rounds per instance before it is handed back (0: 4V + 1024)
  long long max_ticks;     // device-clock ticks (100 MHz) per instance before it is handed back (0: none)
};

void launch_wg_solve(bool rc, int blocks, hipStream_t st, const WgArgs &a);
// Copies n staged entries into ring slots (tail + i) % R, clears their
// results, then publishes them with a release store of tail + n (one
// workgroup; the only writer of tail).
void launch_pk_publish(hipStream_t st, const WgInst *staged, int32_t n, WgInst *ring, int32_t R, int32_t *result,
                       int32_t *tail);

// Sweep kernels: tiles of P lanes (P = 4..64), one workgroup per long-row chunk,
// and the one-thread round control.  rc: rows in the RCSR layout (else BCSR).
void launch_sweep_tile(int P, bool rc, int blocks, hipStream_t st, const Graph &g, const SweepQ &q);
// pass 0: first chunks of long rows, 1: their other chunks, 2: finish rows of pass 1
void launch_sweep_chunk(int pass, bool rc, int blocks, hipStream_t st, const Graph &g, const SweepQ &q);
void launch_sweep_control(hipStream_t st, const SweepCtl &c);
// Full-scan active-vertex queue (Algorithm 2): vertices v < *span with
// e(v) > 0 and h(v) < hcap, appended to list / *cnt.
void launch_avq_scan(int blocks, hipStream_t st, const Graph &g, const int32_t *span, int32_t *list, int32_t *cnt,
                     int32_t cap, int32_t *err, const int32_t *halt);
// Cooperative global relabel (all workgroups co-resident).
hipError_t launch_global_relabel(int P, bool rc, int blocks, hipStream_t st, GRArgs &a);
// Co-resident workgroup limit of the global relabel for P lanes.
int gr_max_blocks(int device, int P);

}  // namespace wb
