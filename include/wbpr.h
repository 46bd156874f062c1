/*
 * wbpr.h -- C ABI of the MI355X (gfx950) workload-balanced push-relabel
 * maximum-flow library.
 *
 * Problem (paper, section 2.1): a directed graph G(V,E) in which every arc
 * (u,v) carries an integer capacity c(u,v) >= 0, a source s and a sink t.
 * The library returns the maximum s-t flow value, one maximum flow (the flow
 * on every input arc) and the canonical minimum cut: side[v] = 1 iff v can
 * still reach t in the residual graph of a maximum flow (the sink side).
 * This set is the same for every maximum flow, so it is bit-comparable.
 *
 * Method (paper, Algorithm 1 and Algorithm 2, sections 2.2 and 3): the
 * lock-free push-relabel algorithm with the vertex-centric two-level
 * parallelism: each sweep compacts the active vertices (e(u) > 0,
 * h(u) < |V|) into an active-vertex queue, a group of lanes scans each queued
 * vertex's residual arcs in the bidirectional CSR (section 3.2) for the
 * minimum-height residual neighbour, and the vertex pushes (atomic updates of
 * residuals and excesses: by default along every residual arc to a lower
 * neighbour while excess is left, push_mode 1 is the paper's single push) or
 * relabels.  A global relabel (backward BFS from the sink in the residual
 * graph, section 2.2) resets heights periodically; it runs on the GPU.
 * Between global relabels a gap heuristic (not in the paper's method; option
 * gap) parks the vertices above an emptied height until the next one.  Small
 * instances alone on the device are solved whole by one workgroup with the
 * residual graph in LDS (wbpr_options.lds_max_v).  Everything is exact integer
 * arithmetic: capacities and residuals int32, excesses and flow values int64.
 *
 * Graph input (all entry points):
 *   row_ptr  int64[V+1], row_ptr[0] = 0, non-decreasing, row_ptr[V] = E
 *   col      int32[E],  0 <= col[i] < V       (arc i = (u, col[i]) for
 *                                               row_ptr[u] <= i < row_ptr[u+1])
 *   cap      int32[E],  cap[i] >= 0
 * Parallel arcs, antiparallel arcs, zero capacities and self-loops are all
 * allowed (a self-loop always carries flow 0).  Limits: 2 <= V < 2^30,
 * E < 2^30, at most 2^31-1 merged residual entries, and for every vertex
 * pair c(u->v) + c(v->u) summed over parallel arcs must fit in int32
 * (WBPR_EOVERFLOW otherwise).
 *
 * Outputs: value int64; arc_flow int32[E] (0 <= f <= cap, conserved at every
 * v not in {s,t}); cut_side uint8[V] (0 = source side, 1 = sink side).
 *
 * Errors: every function returns an int status (WBPR_OK = 0).  On failure
 * wbpr_last_error() gives a message for the calling thread.  No exception
 * or abort crosses the ABI.  Output buffers are unspecified after a failure.
 */
#ifndef WBPR_H
#define WBPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum wbpr_status {
    WBPR_OK = 0,
    WBPR_EINVAL = 1,     /* bad argument or malformed graph */
    WBPR_ENOMEM = 2,     /* device or host allocation failed */
    WBPR_ETOOBIG = 3,    /* graph exceeds a size limit or the admission budget */
    WBPR_ETIMEOUT = 4,   /* max_sweeps / max_wall_ms watchdog fired */
    WBPR_EDEVICE = 5,    /* HIP runtime error */
    WBPR_EAGAIN = 6,     /* result not ready yet (server polling) */
    WBPR_EOVERFLOW = 7,  /* merged pair capacity does not fit in int32 */
    WBPR_EINTERNAL = 8,  /* internal consistency check failed (a bug) */
    WBPR_ECANCELED = 9   /* server request dropped by wbpr_server_destroy */
};

/* Graph in CSR.  Pointers are host or device memory depending on the entry
 * point (see each function).  The caller owns them; the library only reads
 * them during the call (or until the stream work completes for
 * wbpr_solve_device). */
typedef struct wbpr_csr {
    int32_t V;
    int64_t E;
    const int64_t *row_ptr;
    const int32_t *col;
    const int32_t *cap;
} wbpr_csr;

/* Residual-graph layouts (paper, section 3.2; same results, different speed):
 *   BCSR: bidirectional CSR, one entry per ordered vertex pair (parallel and
 *     antiparallel arcs merged), columns sorted, the mate entry of every
 *     entry precomputed; every residual read is coalesced.
 *   RCSR: the input CSR (forward entries, residual c - f) beside a reversed
 *     CSR of every vertex's in-arcs whose entries point at the arc's forward
 *     entry; the residual of a reverse entry (the arc's flow) is read through
 *     that index, one uncoalesced gather.  No merging: parallel arcs stay
 *     separate entries.  Instances in this layout always take the rounds of
 *     launches (no LDS-resident solve).
 * AUTO is BCSR. */
enum wbpr_layout { WBPR_LAYOUT_AUTO = 0, WBPR_LAYOUT_BCSR = 1, WBPR_LAYOUT_RCSR = 2 };

/* Tuning knobs.  Zero means "choose automatically" for every field.  None of
 * them changes the results, only the speed. */
typedef struct wbpr_options {
    int32_t layout;            /* enum wbpr_layout */
    int32_t lanes_per_vertex;  /* lanes scanning one queued vertex: 4,8,16,32,64;
                                  1 = thread-centric: one thread scans a
                                  whole row and, unless split_degree or
                                  block_degree is set, there are no medium
                                  or long tiers (the paper's TC baseline).
                                  0 = automatic: one lane when no row is
                                  longer than 16, else 4, 8 or 16 by the
                                  mean row length */
    int32_t split_degree;      /* rows longer than this get one wave each */
    int32_t gr_every_sweeps;   /* fixed sweeps between global relabels
                                  (0 = adaptive, at most 72) */
    int64_t max_sweeps;        /* watchdog on total sweeps (0 = none) */
    int32_t max_wall_ms;       /* watchdog on wall time (0 = none) */
    int32_t grid_blocks;       /* workgroups per tile-kernel launch of a sweep
                                  (0 = 512, two per compute unit) */
    int32_t time_kernels;      /* 1: time every sweep and global-relabel
                                  launch with HIP events (kernel_ms) */
    int32_t push_mode;         /* 1: one push per visit to the minimum-height
                                  residual neighbour, exactly Algorithms 1-2;
                                  0 or 2: full discharge per visit (push along
                                  every lower residual arc, then relabel) */
    int32_t block_degree;      /* rows longer than this get one workgroup each */
    int32_t gr_work_permille;  /* with gr_every_sweeps = 0: a round of sweeps
                                  ends once relabels since the last global
                                  relabel have scanned this many thousandths
                                  of (V + M) entries (0 = 1000) */
    int32_t no_graph;          /* 1: launch sweeps one by one instead of
                                  replaying a captured hipGraph */
    int32_t avq_mode;          /* active-vertex queue: 0 or 2 incremental
                                  (push targets and still-active vertices are
                                  appended as they go), 1 full scan of every
                                  vertex at the start of each sweep
                                  (Algorithm 2 as printed) */
    int32_t gr_stagnation;     /* with gr_every_sweeps = 0: a round of sweeps
                                  also ends after this many sweeps without a
                                  new smallest active queue (0 = from the mean
                                  row length: 32, 8 or 4 for <= 10, <= 20,
                                  longer) */
    int32_t wave_trace;        /* 1: every wave of every sweep launch records
                                  its execution time and work (the per-warp
                                  timing of the paper's workload analysis,
                                  section 5); read with wbpr_wave_trace */
    int32_t lds_max_v;         /* instances of at most this many vertices
                                  whose residual graph fits one workgroup's
                                  LDS (8 bytes per entry + 20 per vertex,
                                  up to 65,535 of each) are solved whole by
                                  one workgroup at admission, without rounds
                                  of launches (0 = 1024, negative = never) */
    int32_t gap;               /* gap heuristic between global relabels, an
                                  addition to the paper's method (0 or 1 =
                                  on, negative = off): while one instance
                                  runs its phase, relabels keep a count of
                                  vertices at each of the first 256 heights
                                  above its root, and once one of them
                                  empties, sweeps leave every vertex above
                                  it to the next global relabel.  Results
                                  are unchanged */
    int32_t batch_kernel;      /* groups of instances (batches, server
                                  admissions): 0 or 1 = rounds of shared
                                  launches over the disjoint union (a lone
                                  group of small instances is solved in LDS,
                                  see lds_max_v); 2 = every eligible
                                  instance (up to 131,072 vertices and
                                  1,048,576 arcs) by the persistent kernel:
                                  one workgroup per instance, instances
                                  claimed largest first from a device work
                                  queue, each solved whole (exact BFS
                                  heights, sweeps, both phases, flow decode)
                                  with its own tile width and relabel
                                  budget; an instance that reaches a cap
                                  there is finished by the rounds.  The
                                  server with 2 publishes admitted instances
                                  into the running kernel.  The shared
                                  rounds are faster for every size above
                                  the LDS limit, hence the default */
    int32_t debug_checks;      /* 1: before every global relabel (a state
                                  with no sweep running), a check kernel
                                  verifies the invariants of a preflow
                                  (section 2.2) on every instance in the
                                  rounds: no residual capacity is negative;
                                  BCSR: an entry's and its mate's residuals
                                  sum to the pair's capacities; RCSR: an
                                  arc's residual plus its flow is its
                                  capacity and the flow is not negative;
                                  every vertex other than s and t holds
                                  exactly its inflow minus its outflow,
                                  which is not negative.  A violation fails
                                  the call with WBPR_EINTERNAL and a
                                  message with the counts.  Every instance
                                  then takes the rounds of launches (no
                                  LDS-resident or persistent-kernel solve),
                                  so every round is checked; one pass over
                                  the residual graph per round */
} wbpr_options;

/* Per-solve counters and timings (filled when a non-NULL pointer is given). */
typedef struct wbpr_stats {
    int64_t value;
    int64_t V, E, M;               /* vertices, input arcs, merged residual entries */
    int64_t sweeps;                /* sweeps executed (both phases) */
    int64_t global_relabels;       /* global relabels (both phases) */
    int64_t pushes, relabels;      /* push / relabel operations (both phases) */
    int64_t arc_scans;             /* residual entries examined by sweeps */
    int64_t queued;                /* sum of active-queue lengths over sweeps */
    int64_t bfs_scans;             /* entries examined by global relabels */
    int64_t phase2_sweeps;
    int64_t nonempty_sweeps;       /* sweeps that found a non-empty queue */
    int64_t gr_levels;             /* BFS levels summed over global relabels */
    int32_t lanes_per_vertex, split_degree, block_degree, gr_every_sweeps, grid_blocks, gr_blocks;
    double ms_build, ms_phase1, ms_phase2, ms_decode, ms_total;
    /* Per-kernel breakdown.  Index 0: short-row sweep kernel (tiles of
     * lanes_per_vertex lanes), 1: medium-row sweep kernel (one wave per
     * row), 2: long-row sweep kernel (one workgroup per row), 3: global
     * relabel.  kernel_ms / kernel_launches are filled only with
     * time_kernels (HIP events around every launch). */
    double kernel_ms[4];
    int64_t kernel_launches[4];
    int64_t kernel_arc_scans[4];
    int64_t kernel_pushes[4];
    int64_t kernel_relabels[4];
    int64_t kernel_queued[4];
    int64_t bfs_topdown_scans;     /* share of bfs_scans examined top-down */
    int32_t instances;             /* instances solved by the call */
    int32_t use_graph;             /* sweep batches replayed as a hipGraph */
    int64_t lds_solved;            /* instances solved whole in LDS (lds_max_v) */
    int64_t lds_fallbacks;         /* LDS-resident solves that reached their round cap
                                      and were finished by the rounds of launches */
    int64_t gap_skipped;           /* queued vertices the gap heuristic left to the
                                      next global relabel (option gap) */
    double kernel_build_ms;        /* residual-graph builder, device time between
                                      events around it (time_kernels only) */
    int32_t layout;                /* enum wbpr_layout the solve used */
    int32_t reserved0;
    int64_t wg_solved;             /* instances solved by the persistent
                                      workgroup-per-instance kernel */
    int64_t wg_fallbacks;          /* ... that reached a cap there and were
                                      finished by the rounds of launches */
    int64_t debug_checked;         /* rounds whose state passed the invariant
                                      checks (option debug_checks) */
} wbpr_stats;

typedef struct wbpr_ctx wbpr_ctx;

/* Library version string (static storage). */
const char *wbpr_version(void);

/* Message for the last failing call on this thread (static thread-local
 * storage, valid until the next failing call on the same thread). */
const char *wbpr_last_error(void);

/* gcnArchName of device `dev` into buf (NUL-terminated, truncated to n). */
int wbpr_device_arch(int dev, char *buf, size_t n);

/* Create a context on HIP device `device`.  `opt` may be NULL (defaults).
 * The context owns a growable device arena, a stream and pinned staging
 * buffers; it is not thread-safe.  *out receives the handle. */
int wbpr_ctx_create(int device, const wbpr_options *opt, wbpr_ctx **out);
void wbpr_ctx_destroy(wbpr_ctx *ctx);

/* Replace the context's options (NULL restores the defaults). */
int wbpr_ctx_set_options(wbpr_ctx *ctx, const wbpr_options *opt);

/* Solve one instance from HOST memory.  `g` points to host arrays; they are
 * copied to the device before work starts and may be freed after return.
 * value: required; arc_flow (int32[E]) and cut_side (uint8[V]) may be NULL
 * (then the second phase and the decode are skipped).  Synchronous. */
int wbpr_solve(wbpr_ctx *ctx, const wbpr_csr *g, int32_t s, int32_t t, int64_t *value,
               int32_t *arc_flow, uint8_t *cut_side, wbpr_stats *stats);

/* Solve one instance whose CSR arrays are already in DEVICE memory (e.g.
 * torch tensors).  Outputs are DEVICE pointers: dev_value int64[1]
 * (required), dev_arc_flow int32[E] and dev_cut_side uint8[V] (nullable).
 * `stream` is the caller's hipStream_t (NULL = the legacy default stream),
 * for instance torch.cuda.current_stream().cuda_stream: the library runs on
 * its context's own stream, ordered after the work already queued on
 * `stream` (one event), and makes later work on `stream` wait for the
 * results (one event).  The call returns once the results are written (the
 * solver reads small status words back to drive its loop). */
int wbpr_solve_device(wbpr_ctx *ctx, const wbpr_csr *dev_g, int32_t s, int32_t t, void *stream,
                      int64_t *dev_value, int32_t *dev_arc_flow, uint8_t *dev_cut_side,
                      wbpr_stats *stats);

/* Allocation-free variant of wbpr_solve_device, for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, outputs, stream
 * ordering and errors as wbpr_solve_device; `ctx` must have been created
 * beforehand.  Every byte of device memory the solve needs (the arena and
 * the builder's scratch) is carved from one static array of
 * WBPR_NOALLOC_SCRATCH_BYTES (256 MiB) per device, which each device that
 * runs the library holds from its first use until the process ends.  The
 * call allocates no device or pinned memory and creates no stream, event or
 * graph: sweeps are launched one by one, and there is no per-kernel timing
 * or wave trace.  A graph whose arena and builder scratch exceed the array
 * is rejected with WBPR_ETOOBIG (roughly 69 V + 124 E bytes: V = 100k,
 * E = 1.5M fit).  Every call on a device shares that device's array (from
 * any context or thread) and clears it first, so calls that overlap on one
 * device race: the caller serialises them. */
#define WBPR_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int wbpr_solve_device_noalloc(wbpr_ctx *ctx, const wbpr_csr *dev_g, int32_t s, int32_t t, void *stream,
                              int64_t *dev_value, int32_t *dev_arc_flow, uint8_t *dev_cut_side,
                              wbpr_stats *stats);

/* Batched solve: n independent instances of uneven size, resident together
 * in one device arena and solved as a disjoint union, so one sweep and one
 * global relabel serve all of them (the sweep batch is replayed as a captured
 * hipGraph).  Results per instance are exactly those of separate solves.
 *
 * DEVICE variant: the n CSRs are packed back to back in device memory:
 * instance i contributes V[i] + 1 row pointers (local, starting at 0), E[i]
 * columns (local ids 0..V[i]-1) and E[i] capacities.  V, E, s, t are HOST
 * arrays [n] (local s, t).  Outputs are DEVICE arrays packed the same way:
 * dev_values int64[n] (required), dev_flows int32[sum E] and dev_sides
 * uint8[sum V] (nullable).  Limits: sum V < 2^30, 2 * sum E < 2^31.
 * `stream` as for wbpr_solve_device (ordered after its queued work, and
 * later work on it waits for the results); returns once they are written.
 *
 * status (HOST int32[n], nullable): per-instance results.  NULL: any
 * invalid instance fails the whole call with its code.  Non-NULL: an
 * instance that fails its checks (WBPR_EINVAL: sizes, s/t, row pointers,
 * columns, capacities; WBPR_EOVERFLOW: merged capacity over INT32_MAX) gets
 * that code in status[i] and value 0, the others are solved and get
 * WBPR_OK, and the call returns WBPR_OK unless the call itself failed (null
 * arrays, negative sizes, which leave the packing undefined, or a device
 * error).  When an instance fails a device check, the rest are solved one
 * by one and `stats` is zeroed. */
int wbpr_solve_batch_device(wbpr_ctx *ctx, int32_t n, const int32_t *V, const int64_t *E, const int32_t *s,
                            const int32_t *t, const int64_t *dev_row_ptr, const int32_t *dev_col,
                            const int32_t *dev_cap, void *stream, int64_t *dev_values, int32_t *dev_flows,
                            uint8_t *dev_sides, wbpr_stats *stats, int32_t *status);

/* HOST variant: graphs[i] are host CSRs (copied before work starts),
 * s[i], t[i] local; values int64[n] (required); flows (nullable) holds n
 * pointers to int32[E_i]; sides (nullable) holds n pointers to uint8[V_i].
 * status as above (an instance with null arrays is one more WBPR_EINVAL;
 * the flows and sides of a failed instance are left untouched). */
int wbpr_solve_batch(wbpr_ctx *ctx, int32_t n, const wbpr_csr *graphs, const int32_t *s, const int32_t *t,
                     int64_t *values, int32_t *const *flows, uint8_t *const *sides, wbpr_stats *stats,
                     int32_t *status);

/* ------------------------------------------------------------------------
 * Uploaded graphs: build the residual graph once, solve many (s, t) pairs.
 *
 * The residual graph (bidirectional CSR with merged parallel/antiparallel
 * arcs, mates and the arc -> entry map, paper section 3.2) does not depend on
 * s and t.  An uploaded graph keeps it on the device; every solve resets the
 * residual capacities from the stored merged capacities and runs the same
 * path as wbpr_solve without the builder.
 * ---------------------------------------------------------------------- */
typedef struct wbpr_graph wbpr_graph;

/* Upload a host CSR (copied; the caller may free it after return) and build
 * its residual graph on ctx's device with ctx's options (copied).  The
 * handle owns its own stream and device arena (O(V + E), see
 * wbpr_server_footprint); ctx may be destroyed afterwards.  Validation as
 * wbpr_solve (WBPR_EINVAL, WBPR_EOVERFLOW, WBPR_ETOOBIG). */
int wbpr_graph_upload(wbpr_ctx *ctx, const wbpr_csr *g, wbpr_graph **out);

/* Maximum s-t flow on an uploaded graph; outputs as wbpr_solve (host
 * buffers, arc_flow and cut_side nullable).  Synchronous; one solve at a time
 * per handle (not thread-safe).  After a failure other than WBPR_EINVAL the
 * handle is unusable (every later solve fails) and should be freed. */
int wbpr_graph_solve(wbpr_graph *gr, int32_t s, int32_t t, int64_t *value, int32_t *arc_flow, uint8_t *cut_side,
                     wbpr_stats *stats);

void wbpr_graph_free(wbpr_graph *gr);

/* Autotuner: picks the schedule (lanes per vertex, relabel-work budget,
 * stagnation window, queue mode) for graphs shaped like g.  The graph is uploaded once; each
 * candidate schedule solves (s, t) once to warm up and once timed (flows
 * and cut included); every candidate must give the same flow value
 * (WBPR_EINTERNAL otherwise: results never depend on the schedule).  The
 * fastest is written to *best (other fields copied from ctx's options) with
 * its time in *best_ms (nullable), and remembered in ctx for the graph's
 * shape class (log2 V and log2 of the mean row length); later solves on ctx
 * whose options leave lanes_per_vertex and gr_work_permille at 0 use the
 * remembered schedule for graphs of that class.  max_trials bounds the
 * number of candidates (0 = all, at most 20); include_full_scan adds the
 * full-scan queue to the candidates. */
int wbpr_autotune(wbpr_ctx *ctx, const wbpr_csr *g, int32_t s, int32_t t, int32_t max_trials,
                  int32_t include_full_scan, wbpr_options *best, double *best_ms);

/* Per-wave trace of the last solve on ctx (section 5, workload analysis: the
 * paper times every warp from its first thread; here the first lane of every
 * wave of every sweep launch that ran records one entry).  Needs
 * wave_trace = 1 in the options of that solve; else *count = 0.
 * A record is four int32: [0] = sweep index since the solve started * 4 +
 * kernel (0 short-row tiles, 1 medium rows, one wave each, 2 first chunks
 * of long rows, 3 further chunks), [1] the wave's execution time in ticks of
 * the 100 MHz device wall clock (from its first to its last instruction of
 * the launch), [2] residual entries it scanned, [3] vertices (kernels 0-2) or
 * chunk tasks (kernel 3) it processed.  Waves that found nothing to do are
 * recorded too ([3] = 0).  A solve keeps at most 4,194,304 records (the rest
 * are dropped).  Copies min(*count, cap) records into the HOST array
 * records[4 * cap] (nullable when cap = 0); *count = records kept.  Records
 * are in completion order.  WBPR_EINVAL: ctx or count NULL, cap < 0, or
 * records NULL with cap > 0. */
int wbpr_wave_trace(wbpr_ctx *ctx, int32_t *records, int64_t cap, int64_t *count);

/* ------------------------------------------------------------------------
 * Multi-terminal front end: the paper's experimental protocol (section 4).
 * Graphs without given terminals get source/sink pairs chosen by
 * breadth-first search among the vertices farthest apart, and a
 * super-source and a super-sink joined to all of them make the multi-source,
 * multi-sink problem one s-t maximum flow.  BFS distances count arcs of
 * positive capacity (the network at zero flow); self-loops never count.
 * g is a HOST CSR (validated on the host: row pointers, columns in range).
 * ---------------------------------------------------------------------- */

/* Eccentricity of each from[i] (largest BFS distance to a vertex it reaches;
 * 0 when it reaches nothing) into ecc[i], and the farthest vertex (smallest
 * id among those at that distance; from[i] itself when it reaches nothing)
 * into farthest[i].  HOST arrays [n].  Runs on the GPU as a bit-parallel
 * BFS of up to 64 sources per pass (24 bytes per vertex of device memory
 * for the call).  WBPR_ETIMEOUT when the context's max_wall_ms passes. */
int wbpr_bfs_farthest(wbpr_ctx *ctx, const wbpr_csr *g, int32_t n, const int32_t *from, int32_t *ecc,
                      int32_t *farthest);

/* Up to k source/sink pairs by the paper's rule, read as: 4k candidate
 * sources (distinct vertices with an arc of positive capacity to another
 * vertex, drawn by SplitMix64 from `seed`, x -> x mod V in draw order), each
 * paired with its farthest vertex; the pairs are taken by decreasing
 * eccentricity (draw order on ties), skipping pairs with eccentricity 0 or
 * a vertex already used, so the k kept (the top quarter of the candidates
 * when enough are usable) use 2k distinct vertices.  HOST arrays
 * sources[k], sinks[k]; *npairs = pairs written (may be below k). */
int wbpr_pick_terminals(wbpr_ctx *ctx, const wbpr_csr *g, int32_t k, uint64_t seed, int32_t *sources,
                        int32_t *sinks, int32_t *npairs);

/* Maximum flow from the k sources to the k sinks (HOST arrays [k], 2k
 * distinct vertices): a super-source S = V with an arc to every source of
 * that source's outgoing capacity and a super-sink T = V + 1 with an arc
 * from every sink of that sink's incoming capacity (neither can bind) are
 * added, and the s-t path solves (S, T).  Outputs as wbpr_solve, for the
 * original graph: *value, arc_flow[E] and cut_side[V] (HOST, nullable;
 * cut_side[v] = 1 when v reaches T in the final residual graph).  Errors as
 * wbpr_solve; WBPR_EINVAL for a terminal out of range or listed twice;
 * WBPR_EOVERFLOW when a terminal's capacity sum exceeds INT32_MAX. */
int wbpr_solve_multi(wbpr_ctx *ctx, const wbpr_csr *g, int32_t k, const int32_t *sources, const int32_t *sinks,
                     int64_t *value, int32_t *arc_flow, uint8_t *cut_side, wbpr_stats *stats);

/* ------------------------------------------------------------------------
 * Continuous-batching server.
 *
 * Requests (one instance each) arrive at any time from any thread.  A worker
 * thread owns a device arena of fixed capacity, carved from an HBM budget:
 * between rounds it admits waiting requests whose residual graphs fit the
 * free vertex, entry and arc ranges and a free instance slot, and every round
 * runs one multi-root global relabel and one batch of sweeps over everything
 * resident, so requests that arrive while others are solving join the same
 * launches (continuous batching).  Residual state stays on the device until
 * the instance finishes; the result is then copied back and its ranges are
 * returned.  Each result is exactly what a separate solve gives.
 *
 * Admission footprint of one instance with V vertices and E arcs (bytes of
 * the arena it occupies while resident, see wbpr_server_footprint):
 *   69 V + 44 E + ceil(E / 32)
 *     (rows 8V; entries 16 B per slot, 2E slots; arcs 12E; excess, height,
 *      owner, queues, frontiers, long-row list and counters, visit codes 45V;
 *      BFS chunk descriptors 8(V + 2E/1024); long-row chunk tasks
 *      8(V + 2E/1024))
 * plus outputs 8 + 4E + V and, during admission only, the input staging
 * 8(V+1) + 8E and the builder scratch.
 * ---------------------------------------------------------------------- */
typedef struct wbpr_server wbpr_server;

typedef struct wbpr_server_options {
    int64_t hbm_budget_bytes;  /* device bytes for the arena, builder scratch,
                                  input staging and outputs (0 = 1 GiB) */
    int32_t max_slots;         /* resident instances at most (0 = 256) */
    int32_t arcs_per_vertex;   /* expected E/V, proportions the arena (0 = 8) */
    int32_t want_flows;        /* 1: results carry per-arc flows */
    int32_t want_sides;        /* 1: results carry the cut side */
    int32_t max_admit;         /* requests admitted per round (0 = no limit) */
    int32_t reserved[5];
} wbpr_server_options;

/* One finished request.  arc_flow / cut_side are allocated by the library
 * (NULL unless asked for) and released by wbpr_result_free. */
typedef struct wbpr_result {
    uint64_t ticket;
    int32_t status;            /* WBPR_OK or this request's error */
    int32_t V;
    int64_t E;
    int64_t value;
    int32_t *arc_flow;         /* int32[E] */
    uint8_t *cut_side;         /* uint8[V] */
    double latency_ms;         /* submit -> result ready */
    double queue_ms;           /* submit -> admission */
} wbpr_result;

typedef struct wbpr_server_stats {
    int64_t submitted, completed, failed, pending, resident;
    int64_t rounds, admissions, sweeps;
    double busy_ms;            /* wall time with at least one request in flight */
    double solves_per_s;       /* completed / busy time */
    double p50_ms, p99_ms, max_ms;  /* latency over completed requests */
    int64_t arena_bytes, scratch_bytes, staging_bytes, output_bytes;
    int64_t Vcap, Mcap, Ecap;
    int32_t max_slots, peak_resident;
} wbpr_server_stats;

/* Start a server on ctx's device with ctx's options (copied).  The server has
 * its own stream, arena and worker thread; ctx must outlive it and may still
 * be used for plain solves meanwhile.  WBPR_ETOOBIG if the budget cannot hold
 * a minimal arena. */
int wbpr_server_create(wbpr_ctx *ctx, const wbpr_server_options *opt, wbpr_server **out);

/* Queue one instance (host CSR, copied before return; the caller may free it
 * at once).  Checks the CSR on the host (WBPR_EINVAL) and that the instance
 * can ever be admitted under the budget (WBPR_ETOOBIG).  Thread-safe. */
int wbpr_server_submit(wbpr_server *srv, const wbpr_csr *g, int32_t s, int32_t t, uint64_t *ticket);

/* Result of `ticket`: WBPR_OK and *out filled (ownership passes to the caller,
 * the ticket is retired), WBPR_EAGAIN while pending, WBPR_EINVAL for an
 * unknown ticket.  out->status holds the request's own outcome.
 * Thread-safe. */
int wbpr_server_poll(wbpr_server *srv, uint64_t ticket, wbpr_result *out);

/* Like poll, waiting up to timeout_ms (< 0: no limit) for the result. */
int wbpr_server_wait(wbpr_server *srv, uint64_t ticket, int32_t timeout_ms, wbpr_result *out);

void wbpr_result_free(wbpr_result *r);

/* Counters and latency percentiles since creation.  Thread-safe. */
int wbpr_server_get_stats(wbpr_server *srv, wbpr_server_stats *out);

/* Arena bytes an instance of V vertices and E arcs occupies while resident
 * (formula above).  Pure host function. */
int wbpr_server_footprint(int32_t V, int64_t E, int64_t *bytes);

/* Stop the worker: requests not yet finished complete with WBPR_ECANCELED
 * (their results can no longer be fetched); frees everything. */
void wbpr_server_destroy(wbpr_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* WBPR_H */
