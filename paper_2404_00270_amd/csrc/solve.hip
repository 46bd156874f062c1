// Vertex-centric lock-free push-relabel on the bidirectional CSR.
//
// Paper mapping:
//   * preflow (Algorithm 1, step 0): saturate every residual entry of s.
//   * sweep (Algorithm 2): active vertices sit in an active-vertex queue; a
//     tile of P lanes scans the queued vertex's row (parallel reduction,
//     section 3.3).  In the paper's mode the tile finds the residual entry
//     whose head has the minimum height and its first lane pushes
//     min(e(u), c_f(u,v')) with four atomic updates if h(u) > h(v'), or
//     relabels h(u) = h(v') + 1 (Algorithm 1).  In discharge mode the tile
//     pushes along every residual entry whose head is lower than u, in row
//     order, until e(u) is spent, then relabels if excess is left (each such
//     push obeys the relaxed lock-free rule h(u) > h(v), section 2.2).
//     Rows longer than `split_degree` go to a kernel that gives each of them
//     one wave; rows longer than `block_degree` are cut into chunks of CHUNK
//     entries that many workgroups process at once.
//   * global relabel (section 2.2): backward BFS from the sink in the
//     residual graph sets h(v) to the residual distance to t; unreached
//     vertices get the cap and are inactive.  It runs on the GPU as one
//     cooperative kernel with a grid barrier per BFS level and ends by
//     rebuilding the active-vertex queue from a full scan.
//
// The queue between two global relabels is maintained incrementally: a push
// enqueues its target when the target's excess goes from <= 0 to > 0, and a
// vertex re-enqueues itself while it stays active.  Both tests read the value
// returned by the excess atomics, so every active vertex is enqueued exactly
// once per sweep; one tile then owns it, which the lock-free argument needs
// (only the owner lowers e(u) and the residuals of row u).
//
// Heights: hcap marks "inactive / unreached"; hcap + 1 marks the excluded
// terminal (s in the first phase, t in the second).  Terminals' excesses
// carry WB_EXCESS_BIAS so they never test active.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "wb_common.h"
#include "wb_internal.h"
#include "wb_kernels.h"

namespace wb {



// Pushes d along the residual entry with push handle hk (see handle_of) of
// row u into v: the four atomic updates of Algorithm 1 except the decrement
// of e(u), which the caller applies once per visit.  Returns true when v's
// excess crossed from <= 0 to > 0 (v must then be enqueued, if it is not
// above the cap).
template <bool RC>
__device__ __forceinline__ bool push_entry(const Graph &g, int32_t hk, int32_t v, long long d) {
  if (!RC) {
    atomic_add_i32(&g.ent[hk].y, -(int32_t)d);
    atomic_add_i32(&g.ent[g.rev[hk]].y, (int32_t)d);
  } else if (hk >= 0) {  // forward entry: residual down, flow up
    atomic_add_i32(&g.ent[hk].y, -(int32_t)d);
    atomic_add_i32(&g.flow[hk], (int32_t)d);
  } else {  // reverse entry: the arc's flow down, its forward residual up
    atomic_add_i32(&g.flow[~hk], -(int32_t)d);
    atomic_add_i32(&g.ent[~hk].y, (int32_t)d);
  }
  if (v == *g.sink) return false;
  long long oldv = atomic_add_i64(&g.e[v], d);
  return oldv <= 0 && oldv + d > 0;
}

// Counters of a launch: summed per wave, then per workgroup in LDS, then
// added to the workgroup's partial-counter slot (its own cache line: device
// atomics on one address serialise, and every workgroup of every sweep
// launch adding to the same five counters cost thousands of serialised
// atomics per launch), which the control step folds; without slots, to the
// counters themselves.  Every thread of the workgroup calls it, at the end.
__device__ __forceinline__ void flush_stats(const SweepQ &q, int kofs, long long scans, int pushes, int relabels,
                                            long long queued, long long rwork, long long gskips = 0) {
  long long *stats = q.stats + q.sofs + kofs;
  long long *rwork_ctr = q.rwork;
  long long *gskip_ctr = q.gap_skips;
  if (q.part) {
    long long *slot = q.part + (int64_t)(blockIdx.x % PART_SLOTS) * PART_WORDS;
    stats = slot + q.sofs + kofs;
    rwork_ctr = slot + 12;
    gskip_ctr = slot + 13;
  }
  __shared__ unsigned long long s_acc[6];
  scans = (long long)group_sum_i64<WB_WAVE>(scans);
  long long p = group_sum_i64<WB_WAVE>((long long)pushes);
  long long r = group_sum_i64<WB_WAVE>((long long)relabels);
  queued = group_sum_i64<WB_WAVE>(queued);
  rwork = group_sum_i64<WB_WAVE>(rwork);
  gskips = group_sum_i64<WB_WAVE>(gskips);
  if (threadIdx.x < 6) s_acc[threadIdx.x] = 0;
  __syncthreads();
  if (lane() == 0) {
    if (scans) atomicAdd(&s_acc[0], (unsigned long long)scans);
    if (p) atomicAdd(&s_acc[1], (unsigned long long)p);
    if (r) atomicAdd(&s_acc[2], (unsigned long long)r);
    if (queued) atomicAdd(&s_acc[3], (unsigned long long)queued);
    if (rwork) atomicAdd(&s_acc[4], (unsigned long long)rwork);
    if (gskips) atomicAdd(&s_acc[5], (unsigned long long)gskips);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_acc[0]) atomic_add_i64(&stats[0], (long long)s_acc[0]);
    if (s_acc[1]) atomic_add_i64(&stats[1], (long long)s_acc[1]);
    if (s_acc[2]) atomic_add_i64(&stats[2], (long long)s_acc[2]);
    if (s_acc[3]) atomic_add_i64(&stats[3], (long long)s_acc[3]);
    if (s_acc[4]) atomic_add_i64(rwork_ctr, (long long)s_acc[4]);
    if (s_acc[5] && gskip_ctr) atomic_add_i64(gskip_ctr, (long long)s_acc[5]);
  }
}

// Gap heuristic (an addition to the paper's method, single-instance solves):
// the global relabel leaves in gap_hist the number of vertices at each of
// the first gap[2] heights above the root, and every relabel moves its
// vertex from its old height's count to the new one's.  When a count drops
// to zero, no vertex above that height can reach the root through a
// residual path (heights drop by at most one along residual arcs), so the
// lowest such height is kept in gap[0] and sweeps leave the vertices above
// it, with their excess, to the next global relabel, which labels every
// vertex afresh.  Counts race with concurrent relabels; a transient zero
// only parks vertices until that relabel and never changes a result.
//
// A sweep kernel gathers its moves per workgroup in an LDS histogram (the
// relabels of one launch pile onto a few heights: one device atomic each
// would serialise on those counters).  gap_begin clears it (every thread,
// converged) and returns the heights counted, 0 when the heuristic is off.
__device__ __forceinline__ int32_t gap_begin(const Graph &g, int *s_gap, int32_t *gbase) {
  const int32_t gn = g.gap ? min(g.gap[2], GAP_BINS) : 0;
  *gbase = gn > 0 ? g.gap[1] : 0;
  if (gn > 0) {
    for (int32_t d = threadIdx.x; d < GAP_BINS; d += blockDim.x) s_gap[d] = 0;
    __syncthreads();
  }
  return gn;
}

// One relabel from height ho to hn (n = 0: off) ...
__device__ __forceinline__ void gap_move_lds(int *s_gap, int32_t base, int32_t n, int32_t ho, int32_t hn) {
  const int32_t dn = hn - base, dold = ho - base;
  if (dn > 0 && dn < n) atomicAdd(&s_gap[dn], 1);
  if (dold > 0 && dold < n) atomicSub(&s_gap[dold], 1);
}

// ... and add them to the counts once, at the end (every thread, converged).
__device__ __forceinline__ void gap_flush_lds(const Graph &g, const int *s_gap, int32_t base, int32_t n) {
  if (n <= 0) return;
  __syncthreads();
  for (int32_t d = 1 + threadIdx.x; d < n; d += blockDim.x) {
    const int dlt = s_gap[d];
    if (dlt != 0) {
      const int old = atomicAdd(&g.gap_hist[d], dlt);
      if (dlt < 0 && old + dlt <= 0) atomicMin(&g.gap[0], base + d);
    }
  }
}

// Lowest height found empty (heights above it are cut off), hcap if none.
__device__ __forceinline__ int32_t gap_cut(const Graph &g) {
  return g.gap && g.gap[2] > 0 ? atomic_load_i32(&g.gap[0]) : g.hcap;
}

// Per-wave trace record, written by the first lane of every wave at the end
// of a sweep launch when tracing is on (the paper's per-warp timing, section
// 5).  All lanes of the wave call it, converged.
__device__ __forceinline__ void trace_wave(const SweepQ &q, int kind, long long t0, long long scans,
                                           long long items) {
  scans = group_sum_i64<WB_WAVE>(scans);
  items = group_sum_i64<WB_WAVE>(items);
  if (lane() == 0) {
    const long long dt = (long long)wall_clock64() - t0;
    const int32_t slot = atomic_add_i32(q.wtrace_n, 1);
    if (slot < q.wtrace_cap)
      reinterpret_cast<int4 *>(q.wtrace)[slot] =
          make_int4((*q.sweep_no << 2) | kind, (int)min(dt, 0x7fffffffll), (int)min(scans, 0x7fffffffll),
                    (int)min(items, 0x7fffffffll));
  }
}

// End of a sweep (one thread): stop the rest of this round's sweeps once the
// queue is empty or the relabelling done since the last global relabel has
// scanned more than `budget` entries (then fresh exact heights are worth a
// global relabel).  The flag is read at entry by the next sweeps' kernels,
// so every workgroup of a kernel sees the same decision.
// With a sweep log (diagnostics), every sweep that ran appends one record:
// queue in, medium rows, long rows, second-pass chunk tasks, queue out,
// relabel work since the last global relabel (saturated to int32).
__global__ void __launch_bounds__(PART_SLOTS) k_sweep_control(SweepCtl c) {
  if (*c.halt) return;
  static_assert(PART_SLOTS == WB_WAVE, "one lane per partial-counter slot");
  if (c.part) {
    // fold the sweep kernels' per-workgroup partial counters: lane i takes
    // slot i, then one sum per counter over the wave
    long long *slot = c.part + (int64_t)threadIdx.x * PART_WORDS;
    long long x[14];
#pragma unroll
    for (int k = 0; k < 14; k++) x[k] = slot[k];
#pragma unroll
    for (int k = 0; k < 14; k++) slot[k] = 0;
#pragma unroll
    for (int k = 0; k < 14; k++) {
      if (__ballot(x[k] != 0) == 0) continue;  // wave-uniform
      const long long t = group_sum_i64<WB_WAVE>(x[k]);
      if (threadIdx.x == 0) {
        if (k < 12) c.stats[k] += t;
        else if (k == 12) *c.rwork_acc += t;
        else c.stats[15] += t;  // entries left to the relabel by the gap heuristic
      }
    }
  }
  if (threadIdx.x != 0) return;
  const int32_t next = c.scan_cnt ? *c.qin_cnt : *c.qout_cnt;  // full scan: this sweep's queue
  if (c.log) {
    const int32_t i = *c.log_n;
    if (i < c.log_cap) {
      int32_t *r = c.log + 6 * (int64_t)i;
      const long long rw = *c.rwork - *c.rwork_at_gr;
      r[0] = *c.qin_cnt;
      r[1] = *c.mid_cnt;
      r[2] = *c.big_cnt;
      r[3] = *c.task_cnt;
      r[4] = *c.qout_cnt;
      r[5] = rw > 0x7fffffff ? 0x7fffffff : (int32_t)rw;
      *c.log_n = i + 1;
    }
  }
  // stagnation: the queue has not reached a new minimum (by 1/64) for
  // stag_window sweeps, typically excess circulating among vertices that can
  // no longer reach the root; only a global relabel marks it stranded
  bool stagnant = false;
  if (next < c.stag[0] - (c.stag[0] >> 6)) {
    c.stag[0] = next;
    c.stag[1] = 0;
  } else {
    stagnant = ++c.stag[1] > c.stag_window;
  }
  if (next == 0 || stagnant || *c.rwork - *c.rwork_at_gr > *c.budget) *c.halt = 1;
  if (c.scan_cnt) *c.scan_cnt = 0;
  if (c.sweep_no) *c.sweep_no += 1;
}

// Full-scan queue (Algorithm 2's compaction): ballot over a wave, LDS
// staging, one atomic per flush.
__global__ void __launch_bounds__(SWEEP_THREADS) k_avq_scan(Graph g, const int32_t *span, int32_t *list, int32_t *cnt,
                                                            int32_t cap, int32_t *err, const int32_t *halt) {
  __shared__ int s_qbuf[SWEEP_THREADS / WB_WAVE][WB_QBUF];
  __shared__ int s_qcnt[SWEEP_THREADS / WB_WAVE];
  if (*halt) return;
  const int wl = threadIdx.x / WB_WAVE;
  if (lane() == 0) s_qcnt[wl] = 0;
  const WaveQ wq{s_qbuf[wl], &s_qcnt[wl], list, cnt, cap, err};
  const int64_t n = *span;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int32_t hlim = min(gap_cut(g), g.hcap - 1);  // heights above a gap wait for the relabel
  for (int64_t v0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x - lane(); v0 < n; v0 += nth) {  // wave-uniform
    const int64_t v = v0 + lane();
    bool act = false;
    if (v < n) act = g.e[v] > 0 && g.h[v] <= hlim;
    waveq_push(wq, act, (int32_t)v);
  }
  __shared__ int s_off[SWEEP_THREADS / WB_WAVE + 1];
  block_flush<SWEEP_THREADS / WB_WAVE>(wq, s_off);
}

template <int P>
__device__ __forceinline__ unsigned long long shfl_up_group_u64(unsigned long long v, int d) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = (unsigned)__shfl_up((int)lo, d, WB_WAVE);
  hi = (unsigned)__shfl_up((int)hi, d, WB_WAVE);
  return ((unsigned long long)hi << 32) | lo;
}

// Exclusive prefix sum over an aligned group of P lanes; *total gets the
// group sum in every lane.  All P lanes of the group must be active.
template <int P>
__device__ __forceinline__ long long group_excl_scan_i64(long long x, long long *total) {
  const int tl = lane() & (P - 1);
  long long incl = x;
#pragma unroll
  for (int d = 1; d < P; d <<= 1) {
    long long y = (long long)shfl_up_group_u64<P>((unsigned long long)incl, d);
    if (tl >= d) incl += y;
  }
  *total = (long long)shfl_u64((unsigned long long)incl, lane() | (P - 1));
  return incl - x;
}


// Entry k re-read just before a single push (paper mode): its column, push
// handle and current residual (device-scope load).
template <bool RC>
__device__ __forceinline__ void entry_for_push(const Graph &g, int32_t k, int32_t *v, int32_t *hk, int32_t *r) {
  const int2 ck = g.ent[k];
  *v = col_of<RC>(ck);
  *hk = handle_of<RC>(k, ck);
  *r = RC && ck.x < 0 ? atomic_load_i32(&g.flow[ck.y]) : atomic_load_i32(&g.ent[k].y);
}

constexpr int32_t CHUNK_MORE = 1 << 30;  // lr_cnt flag: a chunk left admissible capacity unpushed
// Bias added to e(u) while the chunks of long row u work on it (discharge
// mode): pushes into u then never see e(u) <= 0, so only u's last chunk
// decides whether u is queued again, and the chunks claim excess from e(u)
// itself.  Excesses of non-terminals stay below 2^61 (at most 2^30 arcs of
// capacity below 2^31 leave s).
constexpr long long CHUNK_BIAS = 1ll << 61;

// Defers long row u to the chunk kernel (one lane): resets the vertex's
// per-sweep chunk state and, in discharge mode, biases its excess.  The chunk
// kernel runs after this kernel, so it sees both.
__device__ __forceinline__ void defer_long_row(const SweepQ &q, const Graph &g, int32_t u) {
  q.lr_key[u] = WB_KEY_NONE;
  q.lr_cnt[u] = 0;
  if (q.mode == 1) atomic_add_i64(&g.e[u], CHUNK_BIAS);
}

// One visit of a queued vertex by a tile of P lanes (rows up to
// split_degree).  Paper mode: the tile reduces the packed key
// (height << 32 | row position) over residual entries to its minimum; the
// first lane pushes min(e(u), c_f) to that neighbour if it is lower, else
// relabels to its height + 1.  Discharge mode: the tile walks the row P
// entries at a time and pushes along every residual entry whose head is
// lower than u, handing out e(u) in row order with a prefix sum, stops once
// e(u) is spent, and relabels to 1 + the lowest remaining residual neighbour
// if excess is left.
template <int P, bool RC>
__global__ void __launch_bounds__(SWEEP_THREADS) k_sweep_tile(Graph g, SweepQ q) {
  constexpr int UNROLL = 4;
  constexpr int DEFER_BUF = 128;
  __shared__ int s_qbuf[SWEEP_THREADS / WB_WAVE][WB_QBUF];
  __shared__ int s_mbuf[SWEEP_THREADS / WB_WAVE][DEFER_BUF];
  __shared__ int s_bbuf[SWEEP_THREADS / WB_WAVE][DEFER_BUF];
  __shared__ int s_qcnt[SWEEP_THREADS / WB_WAVE][3];
  __shared__ int s_gap[GAP_BINS];
  const int wl = threadIdx.x / WB_WAVE;
  if (lane() == 0) {
    s_qcnt[wl][0] = 0;
    s_qcnt[wl][1] = 0;
    s_qcnt[wl][2] = 0;
  }
  const WaveQ wq{s_qbuf[wl], &s_qcnt[wl][0], q.qout, q.qout_cnt, q.qcap, q.err};
  const bool defers = q.t_mid != 0x7fffffff;
  const WaveQ wmid{s_mbuf[wl], &s_qcnt[wl][1], q.mid_v, q.mid_cnt, q.qcap, q.err, DEFER_BUF};
  const WaveQ wbig{s_bbuf[wl], &s_qcnt[wl][2], q.big_v, q.big_cnt, q.qcap, q.err, DEFER_BUF};
  if (*q.halt) return;
  const long long wt0 = q.wtrace ? (long long)wall_clock64() : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && q.zero_cnt) {
    *q.zero_cnt = 0;
    *q.zero_a = 0;
    *q.zero_b = 0;
    *q.zero_c = 0;
    if (*q.qin_cnt > 0) atomic_add_i64(&q.stats[13], 1);
  }
  const int32_t n = min(*q.qin_cnt, q.qcap);
  constexpr int TPW = WB_WAVE / P;  // tiles per wave
  // a workgroup whose first tile is past the queue has nothing to visit
  // (short queues leave most of the grid idle; traced runs keep every wave)
  if ((int64_t)blockIdx.x * (SWEEP_THREADS / WB_WAVE) * TPW >= n && !q.wtrace) return;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t wave = (int32_t)(gtid / WB_WAVE);
  const int32_t nwaves = (int32_t)((int64_t)gridDim.x * blockDim.x / WB_WAVE);
  const int sub = lane() / P;
  const int tl = lane() % P;
  const int tbase = lane() & ~(P - 1);
  long long scans = 0, queued = 0, rwork = 0;
  int pushes = 0, relabels = 0, gskips = 0;
  const int32_t gcut = gap_cut(g);
  int32_t gbase;
  const int32_t gn = gap_begin(g, s_gap, &gbase);
  // one row ahead: the tile's next queue entry is read while its current
  // row is scanned, and the next row's bounds, height and excess before the
  // current row's closing atomics (heights change only by the tile that
  // visits the vertex; excess only grows until then, so the early read is a
  // lower bound and the closing atomic returns the true remainder)
  const int32_t stride = nwaves * TPW;
  int32_t pu = 0, phu = 0;
  int2 prb = make_int2(0, 0);
  long long pe0 = 0;
  {
    const int32_t i0 = wave * TPW + sub;
    if (i0 < n) {
      pu = q.qin[i0];
      prb = g.rowb[pu];
      phu = g.h[pu];
      if (tl == 0) pe0 = atomic_load_i64(&g.e[pu]);
    }
  }
  for (int32_t base = wave * TPW; base < n; base += stride) {  // wave-uniform loop
    const int32_t i = base + sub;
    const bool cut = i < n && phu > gcut && phu < g.hcap;  // above a gap: left to the relabel
    const bool valid = i < n && !cut;
    if (cut && tl == 0) gskips++;
    int32_t u = 0, beg = 0, end = 0, hpre = 0;
    long long epre = 0;
    if (valid) {
      u = pu;
      beg = prb.x;
      end = prb.y;
      hpre = phu;
      epre = pe0;
    }
    const int32_t ni = i + stride;
    pu = ni < n ? q.qin[ni] : 0;
    const int32_t deg = end - beg;
    const bool split = valid && deg > q.t_mid;
    const bool scan = valid && !split;
    const bool leader = tl == 0;
    if (defers) {
      waveq_push(wmid, leader && split && deg <= q.t_big, u);
      const bool big = leader && split && deg > q.t_big;
      if (big) defer_long_row(q, g, u);
      waveq_push(wbig, big, u);
    }
    bool app_u = false;
    if (q.mode == 0) {
      unsigned long long key = WB_KEY_NONE;
      if (scan) {
        for (int32_t kb = beg + tl; kb < end; kb += UNROLL * P) {
          int2 cr[UNROLL];
          int32_t rr[UNROLL];
#pragma unroll
          for (int j = 0; j < UNROLL; j++) cr[j] = kb + j * P < end ? g.ent[kb + j * P] : make_int2(0, 0);
#pragma unroll
          for (int j = 0; j < UNROLL; j++) rr[j] = res_of<RC>(g.flow, cr[j]);
#pragma unroll
          for (int j = 0; j < UNROLL; j++) {
            if (rr[j] > 0) {
              const unsigned long long kk =
                  ((unsigned long long)(unsigned)g.h[col_of<RC>(cr[j])] << 32) | (unsigned)(kb + j * P - beg);
              key = kk < key ? kk : key;
            }
          }
        }
      }
      if (ni < n) {
        prb = g.rowb[pu];
        phu = g.h[pu];
        if (tl == 0) pe0 = atomic_load_i64(&g.e[pu]);
      }
      key = group_min<P>(key);
      bool app_v = false;
      int32_t v = 0;
      if (leader && scan) {
        scans += deg;
        queued += 1;
        if (key == WB_KEY_NONE) {
          app_u = true;  // no residual entry visible yet: retry next sweep
        } else {
          const int32_t hmin = (int32_t)(key >> 32);
          const int32_t k = beg + (int32_t)(key & 0xffffffffu);
          if (g.h[u] > hmin) {
            int32_t hk, rk;
            entry_for_push<RC>(g, k, &v, &hk, &rk);
            long long eu = atomic_load_i64(&g.e[u]);
            long long d = eu < (long long)rk ? eu : (long long)rk;
            if (d > 0) {
              app_v = push_entry<RC>(g, hk, v, d) && g.h[v] < g.hcap;
              long long oldu = atomic_add_i64(&g.e[u], -d);
              app_u = oldu - d > 0;
              pushes++;
            } else {
              app_u = eu > 0;
            }
          } else {
            int32_t nh = hmin + 1;
            if (nh > g.hcap) nh = g.hcap;
            g.h[u] = nh;
            gap_move_lds(s_gap, gbase, gn, hpre, nh);
            relabels++;
            rwork += deg;
            app_u = nh < g.hcap;
          }
        }
      }
      waveq_push(wq, q.append && app_v, v);
    } else {
      // full discharge; every lane of a scanning tile iterates the same count
      const int32_t hu = scan ? hpre : 0;
      long long e0 = (scan && leader) ? epre : 0;
      e0 = (long long)shfl_u64((unsigned long long)e0, tbase);
      long long erem = e0;
      unsigned long long key = WB_KEY_NONE;  // lowest residual entry not lower than u
      long long nscan = 0;
      if (scan) {
        // UNROLL slices of P entries per step: their loads and height
        // gathers are issued together, then the slices are discharged in
        // row order
        for (int32_t kb = beg; kb < end && erem > 0; kb += UNROLL * P) {
          int2 cr[UNROLL];
          int32_t rr[UNROLL];
          int32_t hv[UNROLL];
#pragma unroll
          for (int j = 0; j < UNROLL; j++) {
            const int32_t k = kb + j * P + tl;
            cr[j] = k < end ? g.ent[k] : make_int2(0, 0);
          }
#pragma unroll
          for (int j = 0; j < UNROLL; j++) rr[j] = res_of<RC>(g.flow, cr[j]);
#pragma unroll
          for (int j = 0; j < UNROLL; j++) hv[j] = rr[j] > 0 ? g.h[col_of<RC>(cr[j])] : 0;
          // the pushes of all UNROLL slices are issued before any of their
          // returned excesses is needed (queue appends after the loop), so
          // their atomics overlap.  A head whose excess was <= 0 before the
          // push is not being visited with excess this sweep, so its height
          // is still the gathered one, below u's and so below the cap.
          bool apv[UNROLL];
          int32_t vj[UNROLL];
#pragma unroll
          for (int j = 0; j < UNROLL; j++) {
            const int32_t k = kb + j * P + tl;
            long long want = 0;
            int32_t v = 0;
            if (rr[j] > 0) {
              if (hv[j] < hu) {
                want = rr[j];
                v = col_of<RC>(cr[j]);
              } else {
                unsigned long long kk = ((unsigned long long)(unsigned)hv[j] << 32) | (unsigned)(k - beg);
                key = kk < key ? kk : key;
              }
            }
            long long tot;
            const long long before = group_excl_scan_i64<P>(want, &tot);
            long long take = erem - before;
            take = take < 0 ? 0 : (take > want ? want : take);
            apv[j] = false;
            vj[j] = v;
            if (take > 0) {
              apv[j] = push_entry<RC>(g, handle_of<RC>(k, cr[j]), v, take);
              pushes++;
            }
            if (erem > 0 && kb + j * P < end) nscan += P;
            erem -= tot;
          }
#pragma unroll
          for (int j = 0; j < UNROLL; j++) waveq_push(wq, q.append && apv[j], vj[j]);
        }
      }
      if (ni < n) {
        prb = g.rowb[pu];
        phu = g.h[pu];
        if (tl == 0) pe0 = atomic_load_i64(&g.e[pu]);
      }
      key = group_min<P>(key);
      if (leader && scan) {
        scans += nscan < deg ? nscan : deg;
        queued += 1;
        const long long pushed = e0 - (erem > 0 ? erem : 0);
        long long left = e0;
        if (pushed > 0) left = atomic_add_i64(&g.e[u], -pushed) - pushed;
        if (erem > 0) {
          if (key == WB_KEY_NONE) {
            app_u = true;  // nothing residual visible: retry next sweep
          } else {
            int32_t nh = (int32_t)(key >> 32) + 1;
            if (nh > g.hcap) nh = g.hcap;
            g.h[u] = nh;
            gap_move_lds(s_gap, gbase, gn, hpre, nh);
            relabels++;
            rwork += deg;
            app_u = nh < g.hcap;
          }
        } else {
          app_u = left > 0;
        }
      }
    }
    waveq_push(wq, q.append && app_u, u);
  }
  {
    __shared__ int s_off[SWEEP_THREADS / WB_WAVE + 1];
    block_flush<SWEEP_THREADS / WB_WAVE>(wq, s_off);
    if (defers) {
      block_flush<SWEEP_THREADS / WB_WAVE>(wmid, s_off);
      block_flush<SWEEP_THREADS / WB_WAVE>(wbig, s_off);
    }
  }
  flush_stats(q, 0, scans, pushes, relabels, queued, rwork, gskips);
  gap_flush_lds(g, s_gap, gbase, gn);
  if (q.wtrace) trace_wave(q, q.kind, wt0, scans, queued);
}

constexpr int BLK_WAVES = BLK / WB_WAVE;

// Exclusive prefix sum over the workgroup (BLK threads) in thread order;
// *total gets the workgroup sum.  Contains two barriers.
__device__ __forceinline__ long long block_excl_scan_i64(long long x, long long *total, long long *s_wsum) {
  const int w = threadIdx.x / WB_WAVE;
  long long wtot;
  long long before = group_excl_scan_i64<WB_WAVE>(x, &wtot);
  if (lane() == 0) s_wsum[w] = wtot;
  __syncthreads();
  long long off = 0, tot = 0;
#pragma unroll
  for (int j = 0; j < BLK_WAVES; j++) {
    const long long y = s_wsum[j];
    off += j < w ? y : 0;
    tot += y;
  }
  __syncthreads();
  *total = tot;
  return before + off;
}

// Finishes the visit of long row u (one thread): discharge mode removes the
// bias from e(u) and re-enqueues u while it keeps excess, after relabelling
// it (1 + the minimum over the row) when no chunk left admissible capacity
// unpushed; paper mode pushes to the minimum-key neighbour or relabels
// (Algorithm 1).  Sets *app_u / *app_v (and *v) for the caller's queue.
template <bool RC>
__device__ __forceinline__ void finish_long_row(const Graph &g, const SweepQ &q, int32_t u, int2 rb, int32_t hu,
                                                unsigned long long kmin, bool more, bool *app_u, bool *app_v,
                                                int32_t *v, int *pushes, int *relabels, long long *rwork,
                                                int *s_gap, int32_t gbase, int32_t gn) {
  const int32_t deg = rb.y - rb.x;
  if (q.mode == 1) {
    const long long left = atomic_add_i64(&g.e[u], -CHUNK_BIAS) - CHUNK_BIAS;
    if (left > 0) {
      if (more || kmin == WB_KEY_NONE) {
        *app_u = true;  // admissible capacity left, or nothing residual visible: next sweep
      } else {
        int32_t nh = (int32_t)(kmin >> 32) + 1;
        if (nh > g.hcap) nh = g.hcap;
        g.h[u] = nh;
        gap_move_lds(s_gap, gbase, gn, hu, nh);
        (*relabels)++;
        *rwork += deg;
        *app_u = nh < g.hcap;
      }
    }
  } else if (kmin == WB_KEY_NONE) {
    *app_u = true;
  } else {
    const int32_t hmin = (int32_t)(kmin >> 32);
    const int32_t k = rb.x + (int32_t)(kmin & 0xffffffffu);
    if (hu > hmin) {
      const long long e0 = atomic_load_i64(&g.e[u]);
      int32_t hk, rk;
      entry_for_push<RC>(g, k, v, &hk, &rk);
      const long long d = e0 < (long long)rk ? e0 : (long long)rk;
      if (d > 0) {
        *app_v = push_entry<RC>(g, hk, *v, d) && g.h[*v] < g.hcap;
        const long long oldu = atomic_add_i64(&g.e[u], -d);
        *app_u = oldu - d > 0;
        (*pushes)++;
      } else {
        *app_u = e0 > 0;
      }
    } else {
      int32_t nh = hmin + 1;
      if (nh > g.hcap) nh = g.hcap;
      g.h[u] = nh;
      gap_move_lds(s_gap, gbase, gn, hu, nh);
      (*relabels)++;
      *rwork += deg;
      *app_u = nh < g.hcap;
    }
  }
}

// Long rows, cut into chunks of CHUNK entries processed by one workgroup
// each; thread t holds entries 4t .. 4t+3 of its chunk, so thread order is
// row order.  First pass (FIRST): the first chunk of every deferred row.
// Discharge mode: the chunk sums its admissible capacity (residual entries
// whose head is lower than u), claims up to that much from e(u) (one atomic
// subtract of the sum; what exceeds the excess is given back) and pushes the
// claim along those entries in row order.  If the chunk's admissible capacity
// ran out while u still has excess, the rest of the row is needed: the other
// chunks become tasks of the second pass, which many workgroups process at
// once, and a third pass finishes those rows; otherwise the first chunk
// finishes the visit itself (a hub whose excess fits its first chunk costs
// one chunk, not the whole row).  Chunks fold their lowest non-admissible
// residual key into the vertex's minimum and flag unpushed admissible
// capacity, with atomics whose results they do not wait for.  Paper mode:
// the chunks fold the minimum (height, position) key over all residual
// entries of the row; the finish pushes to that neighbour or relabels.
// Second-pass tasks of the long rows whose first chunk did not settle them,
// gathered by the first pass's thread 0 and listed with one atomic on the
// task counter per workgroup (one per row serialised thousands per launch).
constexpr int TASK_BUF = 64;
__device__ __forceinline__ void flush_tasks(const SweepQ &q, const int32_t *tu, const int32_t *tc, int *tn) {
  int32_t tot = 0;
  for (int i = 0; i < *tn; i++) tot += tc[i] - 1;
  if (tot > 0) {
    int32_t base = atomic_add_i32(q.task_cnt, tot);
    if ((long long)base + tot > (long long)q.tcap) {
      atomic_add_i32(q.err, 1);
    } else {
      for (int i = 0; i < *tn; i++)
        for (int32_t cc = 1; cc < tc[i]; cc++, base++) {
          q.task_u[base] = tu[i];
          q.task_c[base] = cc;
        }
    }
  }
  *tn = 0;
}

template <bool FIRST, bool RC>
__global__ void __launch_bounds__(BLK) k_sweep_chunk(Graph g, SweepQ q) {
  constexpr int PER = CHUNK / BLK;
  __shared__ int32_t s_tu[TASK_BUF];  // first pass, thread 0 only: rows ...
  __shared__ int32_t s_tc[TASK_BUF];  // ... and their chunk counts
  int tn = 0;                         // thread 0's count of them
  __shared__ int s_qbuf[BLK_WAVES][WB_QBUF];
  __shared__ int s_qcnt[BLK_WAVES];
  __shared__ long long s_wsum[BLK_WAVES];
  __shared__ unsigned long long s_wmin[BLK_WAVES];
  __shared__ long long s_take;
  __shared__ int s_gap[GAP_BINS];
  if (*q.halt) return;
  const int32_t ntask = FIRST ? min(*q.big_cnt, q.qcap) : min(*q.task_cnt, q.tcap);
  if ((int32_t)blockIdx.x >= ntask && !q.wtrace) return;  // no task for this workgroup
  const long long wt0 = q.wtrace ? (long long)wall_clock64() : 0;
  int32_t gbase;
  const int32_t gn = gap_begin(g, s_gap, &gbase);
  long long tasks = 0;  // per wave, counted by its first lane
  const int w = threadIdx.x / WB_WAVE;
  if (lane() == 0) s_qcnt[w] = 0;
  const WaveQ wq{s_qbuf[w], &s_qcnt[w], q.qout, q.qout_cnt, q.qcap, q.err};
  long long scans = 0, queued = 0, rwork = 0;
  int pushes = 0, relabels = 0;
  for (int32_t task = blockIdx.x; task < ntask; task += gridDim.x) {
    if (lane() == 0) tasks++;
    const int32_t u = FIRST ? q.big_v[task] : q.task_u[task];
    const int32_t c = FIRST ? 0 : q.task_c[task];
    const int2 rb = g.rowb[u];
    const int32_t deg = rb.y - rb.x;
    const int32_t nch = (deg + CHUNK - 1) / CHUNK;
    const int32_t beg = rb.x + c * CHUNK;
    const int32_t end = min(rb.y, beg + CHUNK);
    const int32_t hu = g.h[u];  // written only when u's visit is finished
    const int32_t k0 = beg + PER * (int32_t)threadIdx.x;
    unsigned long long key = WB_KEY_NONE;
    int32_t vv[PER];
    int32_t want[PER];
    int32_t hk[PER];  // push handles (RCSR; BCSR pushes at k0 + j)
    int2 cr[PER];
    int32_t rr[PER];
    long long mine = 0;
#pragma unroll
    for (int j = 0; j < PER; j++) cr[j] = k0 + j < end ? g.ent[k0 + j] : make_int2(0, 0);
#pragma unroll
    for (int j = 0; j < PER; j++) rr[j] = res_of<RC>(g.flow, cr[j]);
#pragma unroll
    for (int j = 0; j < PER; j++) {
      const int32_t k = k0 + j;
      vv[j] = 0;
      want[j] = 0;
      hk[j] = handle_of<RC>(k, cr[j]);
      if (rr[j] > 0) {
        const int32_t c = col_of<RC>(cr[j]);
        const int32_t hv = g.h[c];
        if (q.mode == 1 && hv < hu) {
          want[j] = rr[j];
          vv[j] = c;
          mine += rr[j];
        } else {
          const unsigned long long kk = ((unsigned long long)(unsigned)hv << 32) | (unsigned)(k - rb.x);
          key = kk < key ? kk : key;
        }
      }
    }
    bool short_claim = false;  // (thread 0) admissible capacity left unpushed
    long long after = 0;       // (thread 0) excess of u left after this chunk's claim
    if (q.mode == 1) {
      long long tot;
      const long long before = block_excl_scan_i64(mine, &tot, s_wsum);
      if (threadIdx.x == 0) {
        long long take = 0;
        if (tot > 0) {
          const long long avail = atomic_add_i64(&g.e[u], -tot) - CHUNK_BIAS;
          take = avail < tot ? (avail > 0 ? avail : 0) : tot;
          if (take < tot) atomic_add_i64(&g.e[u], tot - take);
          after = avail - take;
        } else if (FIRST) {
          after = atomic_load_i64(&g.e[u]) - CHUNK_BIAS;
        }
        short_claim = take < tot;
        s_take = take;
      }
      __syncthreads();
      long long rem = s_take - before;  // claim left for this thread's entries, in row order
      // every push is issued before the returned excesses are needed (as in
      // the tile kernel; a head with excess <= 0 before the push keeps the
      // gathered height, below u's)
      bool apv[PER];
#pragma unroll
      for (int j = 0; j < PER; j++) {
        const long long d = rem < 0 ? 0 : (rem > want[j] ? want[j] : rem);
        apv[j] = false;
        if (d > 0) {
          apv[j] = push_entry<RC>(g, RC ? hk[j] : k0 + j, vv[j], d);
          pushes++;
        }
        rem -= want[j];
      }
#pragma unroll
      for (int j = 0; j < PER; j++) waveq_push(wq, q.append && apv[j], vv[j]);
    }
    key = group_min<WB_WAVE>(key);
    if (lane() == 0) s_wmin[w] = key;
    __syncthreads();
    bool app_u = false, app_v = false;
    int32_t v = 0;
    if (threadIdx.x == 0) {
      for (int j = 0; j < BLK_WAVES; j++) key = s_wmin[j] < key ? s_wmin[j] : key;
      scans += end - beg;
      if (FIRST && (nch == 1 || (q.mode == 1 && (short_claim || after <= 0)))) {
        // the first chunk settles the visit alone; its minimum covers the
        // whole row only when the row is one chunk, so a longer row is not
        // relabelled here (excess that arrived meanwhile waits a sweep)
        queued += 1;
        finish_long_row<RC>(g, q, u, rb, hu, key, short_claim || nch > 1, &app_u, &app_v, &v, &pushes, &relabels,
                            &rwork, s_gap, gbase, gn);
      } else {
        if (key != WB_KEY_NONE) atomic_min_u64(&q.lr_key[u], key);
        if (short_claim) atomic_or_i32(&q.lr_cnt[u], CHUNK_MORE);
        if (FIRST) {  // the other chunks become second-pass tasks (listed at the end)
          if (tn == TASK_BUF) flush_tasks(q, s_tu, s_tc, &tn);
          s_tu[tn] = u;
          s_tc[tn] = nch;
          tn++;
        }
      }
    }
    if (w == 0) {
      waveq_push(wq, q.append && app_v, v);
      waveq_push(wq, q.append && app_u, u);
    }
    __syncthreads();  // s_take, s_wmin and s_wsum are reused by the next task
  }
  if (FIRST && threadIdx.x == 0) flush_tasks(q, s_tu, s_tc, &tn);
  {
    __shared__ int s_off[BLK_WAVES + 1];
    block_flush<BLK_WAVES>(wq, s_off);
  }
  flush_stats(q, 8, scans, pushes, relabels, queued, rwork);
  gap_flush_lds(g, s_gap, gbase, gn);
  if (q.wtrace) trace_wave(q, FIRST ? 2 : 3, wt0, scans, tasks);
}

// Third pass: one thread finishes each long row whose chunks ran in the
// second pass (the row's task with chunk index 1 stands for it).
template <bool RC>
__global__ void __launch_bounds__(BLK) k_sweep_chunk_finish(Graph g, SweepQ q) {
  __shared__ int s_qbuf[BLK_WAVES][WB_QBUF];
  __shared__ int s_qcnt[BLK_WAVES];
  __shared__ int s_gap[GAP_BINS];
  if (*q.halt) return;
  const int32_t ntask = min(*q.task_cnt, q.tcap);
  if ((int64_t)blockIdx.x * blockDim.x >= ntask) return;  // no task for this workgroup
  int32_t gbase;
  const int32_t gn = gap_begin(g, s_gap, &gbase);
  const int w = threadIdx.x / WB_WAVE;
  if (lane() == 0) s_qcnt[w] = 0;
  const WaveQ wq{s_qbuf[w], &s_qcnt[w], q.qout, q.qout_cnt, q.qcap, q.err};
  long long queued = 0, rwork = 0;
  int pushes = 0, relabels = 0;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < ntask; b0 += nth) {  // wave-uniform
    const int64_t i = b0 + threadIdx.x;
    bool app_u = false, app_v = false;
    int32_t u = 0, v = 0;
    if (i < ntask && q.task_c[i] == 1) {
      u = q.task_u[i];
      const int2 rb = g.rowb[u];
      queued += 1;
      finish_long_row<RC>(g, q, u, rb, g.h[u], atomic_load_u64(&q.lr_key[u]), (q.lr_cnt[u] & CHUNK_MORE) != 0,
                          &app_u, &app_v, &v, &pushes, &relabels, &rwork, s_gap, gbase, gn);
    }
    waveq_push(wq, q.append && app_v, v);
    waveq_push(wq, q.append && app_u, u);
  }
  {
    __shared__ int s_off[BLK_WAVES + 1];
    block_flush<BLK_WAVES>(wq, s_off);
  }
  flush_stats(q, 8, 0, pushes, relabels, queued, rwork);
  gap_flush_lds(g, s_gap, gbase, gn);
}

// ------------------------------------------------------ global relabel

__device__ __forceinline__ uint8_t dist_code(int32_t d) { return (uint8_t)(1 + (d & 1)); }

__device__ __forceinline__ bool bm_test(const uint32_t *bm, int32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ __forceinline__ void bm_set(uint32_t *bm, int32_t v) {
  __hip_atomic_fetch_or(&bm[v >> 5], 1u << (v & 31), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Running per-wave count for the common case of one key per wave step
// (wave-uniform): flushed with one atomic when the key changes and at the
// end, instead of one atomic per wave step on the same counter.
struct KeyCount {
  int32_t key = -1;
  int32_t cnt = 0;
};

// counters[key] += number of lanes with pred and that key; one atomic per
// distinct key in the wave (consecutive vertices mostly share an instance).
__device__ __forceinline__ void wave_count_by_key(bool pred, int32_t key, int32_t *counters) {
  unsigned long long m = __ballot(pred);
  while (m) {
    const int leader = __ffsll((long long)m) - 1;
    const int32_t k = __shfl(key, leader, WB_WAVE);
    const unsigned long long same = __ballot(pred && key == k);
    if (lane() == leader) atomic_add_i32(&counters[k], __popcll(same));
    m &= ~same;
  }
}

__device__ __forceinline__ void key_count_flush(KeyCount &kc, int32_t *counters) {
  if (kc.cnt && lane() == 0) atomic_add_i32(&counters[kc.key], kc.cnt);
  kc.cnt = 0;
}

__device__ __forceinline__ void key_count_add(bool pred, int32_t key, KeyCount &kc, int32_t *counters) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  const int32_t k0 = __shfl(key, leader, WB_WAVE);
  if (__ballot(pred && key == k0) == m) {
    if (k0 != kc.key) {
      key_count_flush(kc, counters);
      kc.key = k0;
    }
    kc.cnt += __popcll(m);
  } else {
    wave_count_by_key(pred, key, counters);
  }
}

// Global relabel (section 2.2): backward BFS from the root (the sink in the
// first phase, the source in the second) over residual arcs v -> w with
// c_f(v,w) > 0, h(v) = h(w) + 1.  One cooperative launch; a grid barrier
// separates BFS levels.  A level runs top-down (frontier queue; tiles of P
// lanes expand rows, claiming heads by compare-and-swap on h) while the
// frontier is small and bottom-up (every unvisited vertex looks through its
// own row for a residual arc into the frontier, no atomics) once it is large.
// A vertex at distance d carries visit code 1 + (d & 1): an unvisited vertex
// can only have residual arcs into distance-L vertices during step L (one at
// distance L-2 would have made it distance L-1), so "code == code(L)" names
// the frontier exactly.
// Sums (x, y) over the workgroup in LDS; thread 0 adds the nonzero totals
// to the device counters (one atomic per workgroup and counter instead of
// one per wave).  Every thread of the workgroup calls it, converged.
__device__ __forceinline__ void block_add2(int32_t x, long long y, int32_t *cx, long long *cy) {
  __shared__ unsigned long long s2[2];
  x = wave_sum_i32(x);
  y = group_sum_i64<WB_WAVE>(y);
  if (threadIdx.x == 0) {
    s2[0] = 0;
    s2[1] = 0;
  }
  __syncthreads();
  if (lane() == 0) {
    if (x) atomicAdd(&s2[0], (unsigned long long)x);
    if (y) atomicAdd(&s2[1], (unsigned long long)y);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (cx && s2[0]) atomic_add_i32(cx, (int32_t)s2[0]);
    if (s2[1]) atomic_add_i64(cy, (long long)s2[1]);
  }
}

template <int P, bool RC>
__global__ void __launch_bounds__(GR_THREADS) k_global_relabel(GRArgs a) {
  __shared__ int s_qbuf[GR_THREADS / WB_WAVE][WB_QBUF];
  __shared__ int s_qcnt[GR_THREADS / WB_WAVE];
  __shared__ int s_goff[GR_THREADS / WB_WAVE + 1];
  const Graph &g = a.g;
  const unsigned nblocks = gridDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int32_t wave = (int32_t)(gtid / WB_WAVE);
  const int32_t nwaves = (int32_t)(nthreads / WB_WAVE);
  const int wl = threadIdx.x / WB_WAVE;
  constexpr int TPW = WB_WAVE / P;
  const int sub = lane() / P;
  const int tl = lane() % P;
  const int tbase = lane() & ~(P - 1);
  if (lane() == 0) s_qcnt[wl] = 0;

  if (a.tlog && gtid == 0) {
    a.tlog[0] = (long long)wall_clock64();
    a.tlog[1] = -2;  // set-up
    a.tlog[2] = 0;
  }
  for (int64_t v = gtid; v < g.V; v += nthreads) {
    g.h[v] = g.hcap;
    a.vis[v] = 0;
  }
  // gap heuristic: counts per distance from the root, filled level by level
  // below; no gap until a relabel empties one
  for (int64_t j = gtid; j < a.gap_n; j += nthreads) g.gap_hist[j] = 0;  // gap_n <= GAP_BINS
  if (gtid == 0 && g.gap) {
    g.gap[0] = g.hcap;
    g.gap[1] = a.gap_base;
    g.gap[2] = a.gap_n;
  }
  // frontier membership and visited flags as bitmaps (1/32 of a byte array:
  // they stay in L2 where the per-entry gathers of a level hit them)
  uint32_t *const bm_vis = a.bm;
  for (int64_t j = gtid; j < 4 * (int64_t)a.bm_words; j += nthreads) a.bm[j] = 0;
  for (int64_t j = gtid; j < a.nroots; j += nthreads) a.fq[0][j] = a.roots[j];
  for (int64_t j = gtid; j < a.ninst; j += nthreads) {
    a.inst_active[j] = 0;
    a.inst_stranded[j] = 0;
  }
  if (gtid == 0) {
    a.status[0] = 0;
    a.status[1] = 0;
    a.status[2] = 0;
    a.status[3] = 0;
    a.fcnt[0] = a.nroots;
    a.fcnt[1] = 0;
    a.fcnt[2] = 0;
    a.chunk_cnt[0] = 0;
    a.chunk_cnt[1] = 0;
    a.bucnt[0] = 0;
    a.bucnt[1] = 0;
    a.bucnt[2] = 0;
    a.fedges[0] = 0;
    a.fedges[1] = 0;
    a.fedges[2] = 0;
    a.qcnt[0] = 0;
    a.qcnt[1] = 0;
    a.qcnt[2] = 0;
    a.big_cnt[0] = 0;
    a.big_cnt[1] = 0;
    a.mid_cnt[0] = 0;
    a.mid_cnt[1] = 0;
    a.task_cnt[0] = 0;
    a.task_cnt[1] = 0;
  }
  grid_barrier(a.bar, nblocks);
  long long root_edges = 0;
  for (int64_t j = gtid; j < a.nroots; j += nthreads) {
    g.h[a.roots[j]] = a.root_h[j];
    a.vis[a.roots[j]] = dist_code(0);
    bm_set(bm_vis, a.roots[j]);
    bm_set(a.bm + a.bm_words, a.roots[j]);  // frontier of level 0
    const int2 rb = g.rowb[a.roots[j]];
    root_edges += rb.y - rb.x;
  }
  // row lengths of the roots: a root whose row holds a large share of the
  // entries (the grid cut's sink) is expanded bottom-up from level 0
  root_edges = group_sum_i64<WB_WAVE>(root_edges);
  if (lane() == 0 && root_edges) atomic_add_i64(&a.fedges[0], root_edges);
  for (int64_t j = gtid; j < a.nexcl; j += nthreads) {
    g.h[a.excl[j]] = g.hcap + 1;
    a.vis[a.excl[j]] = 3;
    bm_set(bm_vis, a.excl[j]);
  }
  grid_barrier(a.bar, nblocks);

  long long bscans = 0, buscans = 0;  // entries examined top-down / bottom-up
  int32_t level = 0, bu_levels = 0;
  int32_t n = min(a.nroots, a.qcap);
  long long nedges = atomic_load_i64(&a.fedges[0]);  // row-length sum of the current frontier
  long long vedges = 0;  // row-length sum of every vertex labelled so far
  bool queue_valid = true;  // the frontier of this level is in fq[level & 1]
  for (;;) {
    if (n == 0) break;
    if (gtid == 0 && level < a.gap_n) g.gap_hist[level] = n;  // the n vertices at distance `level`
    const uint8_t cur = dist_code(level), nxt = dist_code(level + 1);
    // frontier bitmaps rotate over three: this level reads bm_in, writes
    // bm_out (cleared during the previous level) and clears the third
    const uint32_t *bm_in = a.bm + (int64_t)(1 + level % 3) * a.bm_words;
    uint32_t *bm_out = a.bm + (int64_t)(1 + (level + 1) % 3) * a.bm_words;
    uint32_t *bm_clr = a.bm + (int64_t)(1 + (level + 2) % 3) * a.bm_words;
    for (int64_t j = gtid; j < a.bm_words; j += nthreads) bm_clr[j] = 0;
    int32_t *fout = a.fq[(level + 1) & 1];
    int32_t *fout_cnt = &a.fcnt[(level + 1) % 3];
    long long *fe_out = &a.fedges[(level + 1) % 3];
    long long my_edges = 0;  // row lengths of the vertices this thread labels
    if (gtid == 0) {
      a.fcnt[(level + 2) % 3] = 0;
      a.chunk_cnt[(level + 1) & 1] = 0;
      a.bucnt[(level + 2) % 3] = 0;
      a.fedges[(level + 2) % 3] = 0;
    }
    // direction: bottom-up while the frontier is large or its rows hold more
    // than 1/16 of the rows still unvisited (late levels whose frontier is a
    // few hubs are cheaper bottom-up: little is left to scan)
    vedges += nedges;
    const long long unvisited_edges = a.m_total - vedges;
    const bool bottom_up = n > a.bu_threshold || nedges > a.bu_edges || 16 * nedges > unvisited_edges;
    if (a.tlog && gtid == 0 && level + 1 < a.tlog_cap) {
      a.tlog[3 * (level + 1)] = (long long)wall_clock64();
      a.tlog[3 * (level + 1) + 1] = n;
      a.tlog[3 * (level + 1) + 2] = bottom_up ? -nedges - 1 : nedges;  // sign: direction
    }
    if (bottom_up) {
      bu_levels++;
      // every unvisited vertex looks for a residual arc into the frontier
      // and stops at the first: one lane per vertex (coalesced visit codes
      // and row bounds, most rows are short); rows longer than BU_SHORT are
      // then taken one at a time by the whole wave (the wave's own list, no
      // global step); rows longer than split_deg become chunks
      constexpr int32_t BU_SHORT = 32;
      int found_cnt = 0;
      int32_t *ccnt = &a.chunk_cnt[level & 1];
      // the visit code and row bounds of the wave's next 64 vertices are
      // loaded while the current ones are scanned (only this wave labels
      // them during this pass, and row bounds never change)
      const int64_t bstride = (int64_t)nwaves * WB_WAVE;
      uint8_t nvis = 1;
      int2 nrb = make_int2(0, 0);
      {
        const int64_t v = (int64_t)wave * WB_WAVE + lane();
        if (v < g.V) {
          nvis = a.vis[v];
          nrb = g.rowb[v];
        }
      }
      for (int64_t vb = (int64_t)wave * WB_WAVE; vb < g.V; vb += bstride) {  // wave-uniform
        const int64_t v = vb + lane();
        bool mine = v < g.V && nvis == 0;
        int32_t beg = 0, end = 0;
        if (mine) {
          beg = nrb.x;
          end = nrb.y;
        }
        if (v + bstride < g.V) {
          nvis = a.vis[v + bstride];
          nrb = g.rowb[v + bstride];
        }
        const int32_t deg = end - beg;
        // every row first gets its first BU_SHORT entries examined by its
        // own lane, four per step (their loads and bitmap probes overlap),
        // up to the first residual arc into the frontier: next to a large
        // frontier most vertices are settled here, whatever their row length
        int32_t hitw = -1;
        if (mine) {
          const int32_t pend = end < beg + BU_SHORT ? end : beg + BU_SHORT;
          int32_t k = beg;
          // entries are read in 16-byte pairs from an even index: lanes read
          // different rows, so every load instruction touches 64 cache lines,
          // and pairs halve those requests (a pair's first entry may belong to
          // the row before, which is in bounds and masked out)
          while (k < pend && hitw < 0) {
            const int32_t p0 = k & ~1;
            int2 cr[4];
#pragma unroll
            for (int h2 = 0; h2 < 2; h2++) {
              const int32_t p = p0 + 2 * h2;
              int4 pr = make_int4(0, 0, 0, 0);
              if (p + 1 < end) {
                pr = *reinterpret_cast<const int4 *>(g.ent + p);
              } else if (p < end) {
                const int2 e1 = g.ent[p];
                pr = make_int4(e1.x, e1.y, 0, 0);
              }
              cr[2 * h2] = make_int2(pr.x, pr.y);
              cr[2 * h2 + 1] = make_int2(pr.z, pr.w);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
              const bool in = p0 + j >= k && p0 + j < pend;
              if (hitw < 0 && in && res_of<RC>(g.flow, cr[j]) > 0 && bm_test(bm_in, col_of<RC>(cr[j])))
                hitw = col_of<RC>(cr[j]);
            }
            k = p0 + 4;
          }
          buscans += (k < pend ? k : pend) - beg;
          if (hitw >= 0) {
            g.h[v] = g.h[hitw] + 1;
            a.vis[v] = nxt;
            found_cnt++;
            my_edges += deg;
          }
        }
        // the wave's 64 vertices fill two bitmap words: their bits are set
        // with one atomic per word at the end of the batch, not one per lane
        unsigned long long newbits = __ballot(hitw >= 0);
        // the rest of a longer row without a hit: up to split_deg entries by
        // the whole wave (below), more as chunks of one wave each (next phase)
        const int32_t rbeg = beg + BU_SHORT;
        const bool rest = mine && hitw < 0 && end > rbeg;
        if (rest && end - rbeg > a.split_deg) {
          const int32_t nch = (end - rbeg + a.chunk - 1) / a.chunk;
          const int32_t c0 = atomic_add_i32(ccnt, nch);
          if (c0 + nch <= a.chunk_cap) {
            for (int32_t j = 0; j < nch; j++) {
              a.chunk_w[c0 + j] = (int32_t)v;
              a.chunk_b[c0 + j] = rbeg + j * a.chunk;
            }
          } else {
            atomic_add_i32(a.err, 1);
          }
        }
        // medium rests of this wave, one after the other with all lanes
        unsigned long long med = __ballot(rest && end - rbeg <= a.split_deg);
        while (med) {
          const int src = __ffsll((long long)med) - 1;
          med &= med - 1;
          const int32_t mv = (int32_t)(vb + src);
          const int32_t mb = __shfl(rbeg, src, WB_WAVE), me = __shfl(end, src, WB_WAVE);
          const int32_t mdeg = __shfl(deg, src, WB_WAVE);
          for (int32_t kb = mb; kb < me; kb += WB_WAVE) {  // wave-uniform
            const int32_t k = kb + lane();
            bool hit = false;
            int32_t w = 0;
            if (k < me) {
              const int2 cr = g.ent[k];
              w = col_of<RC>(cr);
              hit = res_of<RC>(g.flow, cr) > 0 && bm_test(bm_in, w);
            }
            const unsigned long long m = __ballot(hit);
            if (lane() == 0) buscans += min(WB_WAVE, me - kb);
            if (m) {
              if (lane() == __ffsll((long long)m) - 1) {
                g.h[mv] = g.h[w] + 1;
                a.vis[mv] = nxt;
                found_cnt++;
                my_edges += mdeg;
              }
              newbits |= 1ull << src;
              break;
            }
          }
        }
        if (newbits && lane() < 2) {  // vb is a multiple of 64
          const unsigned word = (unsigned)(newbits >> (32 * lane()));
          if (word) {
            const int64_t wi = (vb >> 5) + lane();
            __hip_atomic_fetch_or(&bm_vis[wi], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_or(&bm_out[wi], word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      // publish this phase's counts before the barrier
      block_add2(found_cnt, my_edges, &a.bucnt[(level + 1) % 3], fe_out);
      found_cnt = 0;
      my_edges = 0;
      grid_barrier(a.bar, nblocks);
      // long unvisited rows: one wave per chunk; a hit claims v by CAS.
      // nc is read after the barrier, so every workgroup agrees on it and on
      // whether the second barrier below is needed.
      // four wave widths per step: their entry loads and bitmap probes are
      // in flight together (rows that reach this phase mostly hold no
      // residual arc into the frontier and are read to their end); a chunk
      // whose vertex an earlier chunk has labelled is skipped
      const int32_t nc = min(atomic_load_i32(ccnt), a.chunk_cap);
      for (int32_t c = wave; c < nc; c += nwaves) {
        const int32_t v = a.chunk_w[c];
        const int32_t cb = a.chunk_b[c];
        const int2 vrb = g.rowb[v];
        const int32_t ce = min(cb + a.chunk, vrb.y);
        if (bm_test(bm_vis, v)) continue;  // wave-uniform
        constexpr int BU_UNROLL = 4;
        for (int32_t kb = cb; kb < ce; kb += BU_UNROLL * WB_WAVE) {  // wave-uniform
          int2 cr[BU_UNROLL];
#pragma unroll
          for (int j = 0; j < BU_UNROLL; j++) {
            const int32_t k = kb + j * WB_WAVE + lane();
            cr[j] = k < ce ? g.ent[k] : make_int2(0, 0);
          }
          bool hit[BU_UNROLL];
#pragma unroll
          for (int j = 0; j < BU_UNROLL; j++) {
            const int32_t k = kb + j * WB_WAVE + lane();
            hit[j] = k < ce && res_of<RC>(g.flow, cr[j]) > 0 && bm_test(bm_in, col_of<RC>(cr[j]));
          }
          unsigned long long m = 0;
          int32_t w = 0;
#pragma unroll
          for (int j = 0; j < BU_UNROLL; j++) {  // the first hit in row order
            const unsigned long long mj = __ballot(hit[j]);
            if (m == 0 && mj != 0) {
              m = mj;
              w = col_of<RC>(cr[j]);
            }
          }
          if (lane() == 0) buscans += min(BU_UNROLL * WB_WAVE, ce - kb);
          if (m) {
            if (lane() == __ffsll((long long)m) - 1) {
              if (atomicCAS(&g.h[v], g.hcap, g.h[w] + 1) == g.hcap) {
                a.vis[v] = nxt;
                bm_set(bm_vis, v);
                bm_set(bm_out, v);
                found_cnt++;
                my_edges += vrb.y - vrb.x;
              }
            }
            break;
          }
        }
      }
      if (nc > 0) {
        block_add2(found_cnt, my_edges, &a.bucnt[(level + 1) % 3], fe_out);
        grid_barrier(a.bar, nblocks);
      }
      n = min(atomic_load_i32(&a.bucnt[(level + 1) % 3]), a.qcap);
      nedges = atomic_load_i64(fe_out);
      queue_valid = false;
    } else {
      const int32_t *fin = a.fq[level & 1];
      if (!queue_valid) {
        // the frontier was produced bottom-up: list it from its bitmap (the
        // visit codes tell distance parity only, which would also list the
        // vertices two levels back)
        WaveQ wq{s_qbuf[wl], &s_qcnt[wl], a.fq[level & 1], &a.fcnt[level % 3], a.qcap, a.err};
        if (gtid == 0) a.fcnt[level % 3] = 0;
        grid_barrier(a.bar, nblocks);
        for (int64_t v0 = gtid - lane(); v0 < g.V; v0 += nthreads) {
          const int64_t v = v0 + lane();
          waveq_push(wq, v < g.V && bm_test(bm_in, (int32_t)v), (int32_t)v);
        }
        block_flush<GR_THREADS / WB_WAVE>(wq, s_goff);
        grid_barrier(a.bar, nblocks);
        n = min(atomic_load_i32(&a.fcnt[level % 3]), a.qcap);
      }
      WaveQ wq{s_qbuf[wl], &s_qcnt[wl], fout, fout_cnt, a.qcap, a.err};
      int32_t *ccnt = &a.chunk_cnt[level & 1];
      // phase A: tiles of P lanes expand short rows, long rows become chunks
      for (int32_t base = wave * TPW; base < n; base += nwaves * TPW) {
        const int32_t i = base + sub;
        if (i < n) {
          const int32_t w = fin[i];
          const int2 rb = g.rowb[w];
          const int32_t beg = rb.x, end = rb.y;
          const int32_t deg = end - beg;
          if (deg > a.split_deg) {
            if (tl == 0) {
              const int32_t nch = (deg + a.chunk - 1) / a.chunk;
              const int32_t c0 = atomic_add_i32(ccnt, nch);
              if (c0 + nch <= a.chunk_cap) {
                for (int32_t j = 0; j < nch; j++) {
                  a.chunk_w[c0 + j] = w;
                  a.chunk_b[c0 + j] = beg + j * a.chunk;
                }
              } else {
                atomic_add_i32(a.err, 1);
              }
            }
          } else {
            const int32_t hw1 = g.h[w] + 1;
            if (tl == 0) bscans += deg;
            for (int32_t k = beg + tl; k < end; k += P) {
              const int2 cr = g.ent[k];
              const int32_t v = col_of<RC>(cr);
              bool claimed = false;
              if (!bm_test(bm_vis, v) && mate_res<RC>(g.ent, g.rev, g.flow, k, cr) > 0) {
                claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
                if (claimed) {
                  a.vis[v] = nxt;
                  bm_set(bm_vis, v);
                  bm_set(bm_out, v);
                  my_edges += (g.rowb[v].y - g.rowb[v].x);
                }
              }
              waveq_push(wq, claimed, v);
            }
          }
        }
      }
      block_flush<GR_THREADS / WB_WAVE>(wq, s_goff);
      block_add2(0, my_edges, nullptr, fe_out);
      my_edges = 0;
      grid_barrier(a.bar, nblocks);
      // phase B: the chunks of long rows, cut into pieces of one wave's
      // width that all waves take at once (a hub's row is spread over the
      // whole grid; skipped, with its barrier, when the level met no long
      // row: nc is read after the barrier)
      const int32_t nc = min(atomic_load_i32(ccnt), a.chunk_cap);
      const int32_t pieces = (a.chunk + WB_WAVE - 1) / WB_WAVE;
      for (int64_t pc = wave; pc < (int64_t)nc * pieces; pc += nwaves) {
        const int32_t c = (int32_t)(pc / pieces);
        const int32_t w = a.chunk_w[c];
        const int32_t cb = a.chunk_b[c] + (int32_t)(pc % pieces) * WB_WAVE;
        const int32_t ce = min(min(cb + WB_WAVE, a.chunk_b[c] + a.chunk), g.rowb[w].y);
        const int32_t hw1 = g.h[w] + 1;
        if (lane() == 0 && ce > cb) bscans += ce - cb;
        for (int32_t k = cb + lane(); k < ce; k += WB_WAVE) {
          const int2 cr = g.ent[k];
          const int32_t v = col_of<RC>(cr);
          bool claimed = false;
          if (!bm_test(bm_vis, v) && mate_res<RC>(g.ent, g.rev, g.flow, k, cr) > 0) {
            claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
            if (claimed) {
              a.vis[v] = nxt;
              bm_set(bm_vis, v);
              bm_set(bm_out, v);
              my_edges += (g.rowb[v].y - g.rowb[v].x);
            }
          }
          waveq_push(wq, claimed, v);
        }
      }
      if (nc > 0) {
        block_flush<GR_THREADS / WB_WAVE>(wq, s_goff);
        block_add2(0, my_edges, nullptr, fe_out);
        grid_barrier(a.bar, nblocks);
      }
      n = min(atomic_load_i32(fout_cnt), a.qcap);
      nedges = atomic_load_i64(fe_out);
      queue_valid = true;
    }
    level++;
  }
  if (a.tlog && gtid == 0 && level + 1 < a.tlog_cap) {
    a.tlog[3 * (level + 1)] = (long long)wall_clock64();
    a.tlog[3 * (level + 1) + 1] = -1;  // queue rebuild starts
    a.tlog[3 * (level + 1) + 2] = 0;
  }
  // rebuild the active-vertex queue; count, per instance, the active
  // vertices and the excess stranded away from the root
  int stranded = 0;
  {
    WaveQ wq{s_qbuf[wl], &s_qcnt[wl], a.qout, &a.qcnt[0], a.qcap, a.err};
    KeyCount kc_act, kc_str;
    // a wave takes 4 x 64 consecutive vertices at a time: their excess and
    // height loads are all in flight before the first is used
    constexpr int RB = 4;
    for (int64_t v0 = (gtid - lane()) * RB; v0 < g.V; v0 += nthreads * RB) {  // wave-uniform
      long long ev[RB];
      int32_t hv[RB];
#pragma unroll
      for (int j = 0; j < RB; j++) {
        const int64_t v = v0 + j * WB_WAVE + lane();
        ev[j] = v < g.V ? g.e[v] : 0;
        hv[j] = v < g.V ? g.h[v] : 0;
      }
#pragma unroll
      for (int j = 0; j < RB; j++) {
        const int64_t v = v0 + j * WB_WAVE + lane();
        const bool act = ev[j] > 0 && hv[j] < g.hcap;
        const bool str = ev[j] > 0 && hv[j] == g.hcap;
        const int32_t ins = act || str ? a.inst_of[v] : -1;
        stranded += str ? 1 : 0;
        key_count_add(act && ins >= 0, ins, kc_act, a.inst_active);
        key_count_add(str && ins >= 0, ins, kc_str, a.inst_stranded);
        waveq_push(wq, act, (int32_t)v);
      }
    }
    // per-instance counts and the queue tail of every wave, combined over
    // the workgroup before their atomics (the active count of a single
    // instance and the queue counter are one address each)
    __shared__ int32_t s_kk[GR_THREADS / WB_WAVE][4];
    if (lane() == 0) {
      s_kk[wl][0] = kc_act.cnt ? kc_act.key : -1;
      s_kk[wl][1] = kc_act.cnt;
      s_kk[wl][2] = kc_str.cnt ? kc_str.key : -1;
      s_kk[wl][3] = kc_str.cnt;
    }
    __syncthreads();
    if (threadIdx.x < 2) {  // thread 0: active counts, thread 1: stranded counts
      int32_t *ctr = threadIdx.x == 0 ? a.inst_active : a.inst_stranded;
      int32_t key = -1, cnt = 0;
      for (int w = 0; w < GR_THREADS / WB_WAVE; w++) {
        const int32_t k = s_kk[w][2 * threadIdx.x], c = s_kk[w][2 * threadIdx.x + 1];
        if (k < 0) continue;
        if (k != key) {
          if (cnt) atomic_add_i32(&ctr[key], cnt);
          key = k;
          cnt = 0;
        }
        cnt += c;
      }
      if (cnt) atomic_add_i32(&ctr[key], cnt);
    }
    // queue tails: one atomic for the workgroup, then each wave copies its
    // LDS slice to its share
    __shared__ int32_t s_qoff[GR_THREADS / WB_WAVE + 1];
    if (threadIdx.x == 0) {
      int32_t tot = 0;
      for (int w = 0; w < GR_THREADS / WB_WAVE; w++) {
        s_qoff[w] = tot;
        tot += s_qcnt[w];
      }
      s_qoff[GR_THREADS / WB_WAVE] = tot ? atomic_add_i32(&a.qcnt[0], tot) : 0;
    }
    __syncthreads();
    {
      const int32_t c = s_qcnt[wl];
      const int32_t base = s_qoff[GR_THREADS / WB_WAVE] + s_qoff[wl];
      for (int32_t j = lane(); j < c; j += WB_WAVE) {
        const int32_t idx = base + j;
        if (idx < a.qcap) a.qout[idx] = s_qbuf[wl][j];
        else atomic_add_i32(a.err, 1);
      }
    }
  }
  // counters summed over the workgroup first: one atomic per workgroup and
  // counter (one per wave would serialise thousands on each address)
  {
    __shared__ long long s_cnt[3];
    const long long st = wave_sum_i32(stranded);
    const long long bs = group_sum_i64<WB_WAVE>(bscans);
    const long long bus = group_sum_i64<WB_WAVE>(buscans);
    if (threadIdx.x < 3) s_cnt[threadIdx.x] = 0;
    __syncthreads();
    if (lane() == 0) {
      if (st) atomicAdd((unsigned long long *)&s_cnt[0], (unsigned long long)st);
      if (bs) atomicAdd((unsigned long long *)&s_cnt[1], (unsigned long long)bs);
      if (bus) atomicAdd((unsigned long long *)&s_cnt[2], (unsigned long long)bus);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (s_cnt[0]) atomic_add_i64(&a.status[1], s_cnt[0]);
      if (s_cnt[1]) atomic_add_i64(&a.stats[12], s_cnt[1]);
      if (s_cnt[2]) atomic_add_i64(&a.stats[14], s_cnt[2]);
    }
  }
  grid_barrier(a.bar, nblocks);
  if (gtid == 0) {
    if (a.tlog && level + 2 < a.tlog_cap) a.tlog[3 * (level + 2)] = (long long)wall_clock64();
    a.status[0] = a.qcnt[0];
    a.status[2] = level;
    a.status[3] = bu_levels;
    *a.halt = 0;
    *a.rwork_at_gr = *a.rwork;
    a.stag[0] = 0x7fffffff;
    a.stag[1] = 0;
  }
}

// ------------------------------------------------------------ launchers
typedef void (*TileFn)(Graph, SweepQ);
typedef void (*GRFn)(GRArgs);

template <bool RC>
static TileFn tile_fn_rc(int P) {
  switch (P) {
    case 1: return k_sweep_tile<1, RC>;
    case 4: return k_sweep_tile<4, RC>;
    case 8: return k_sweep_tile<8, RC>;
    case 16: return k_sweep_tile<16, RC>;
    case 32: return k_sweep_tile<32, RC>;
    default: return k_sweep_tile<64, RC>;
  }
}
template <bool RC>
static GRFn gr_fn_rc(int P) {
  switch (P) {
    case 4: return k_global_relabel<4, RC>;
    case 8: return k_global_relabel<8, RC>;
    case 16: return k_global_relabel<16, RC>;
    case 32: return k_global_relabel<32, RC>;
    default: return k_global_relabel<64, RC>;
  }
}
static TileFn tile_fn(int P, bool rc) { return rc ? tile_fn_rc<true>(P) : tile_fn_rc<false>(P); }
static GRFn gr_fn(int P, bool rc) { return rc ? gr_fn_rc<true>(P) : gr_fn_rc<false>(P); }

void launch_sweep_tile(int P, bool rc, int blocks, hipStream_t st, const Graph &g, const SweepQ &q) {
  hipLaunchKernelGGL(tile_fn(P, rc), dim3(blocks), dim3(SWEEP_THREADS), 0, st, g, q);
}

void launch_sweep_chunk(int pass, bool rc, int blocks, hipStream_t st, const Graph &g, const SweepQ &q) {
  if (pass == 0) {
    if (rc) hipLaunchKernelGGL((k_sweep_chunk<true, true>), dim3(blocks), dim3(BLK), 0, st, g, q);
    else hipLaunchKernelGGL((k_sweep_chunk<true, false>), dim3(blocks), dim3(BLK), 0, st, g, q);
  } else if (pass == 1) {
    if (rc) hipLaunchKernelGGL((k_sweep_chunk<false, true>), dim3(blocks), dim3(BLK), 0, st, g, q);
    else hipLaunchKernelGGL((k_sweep_chunk<false, false>), dim3(blocks), dim3(BLK), 0, st, g, q);
  } else {
    if (rc) hipLaunchKernelGGL(k_sweep_chunk_finish<true>, dim3(blocks), dim3(BLK), 0, st, g, q);
    else hipLaunchKernelGGL(k_sweep_chunk_finish<false>, dim3(blocks), dim3(BLK), 0, st, g, q);
  }
}

void launch_avq_scan(int blocks, hipStream_t st, const Graph &g, const int32_t *span, int32_t *list, int32_t *cnt,
                     int32_t cap, int32_t *err, const int32_t *halt) {
  hipLaunchKernelGGL(k_avq_scan, dim3(blocks), dim3(SWEEP_THREADS), 0, st, g, span, list, cnt, cap, err, halt);
}

void launch_sweep_control(hipStream_t st, const SweepCtl &c) {
  hipLaunchKernelGGL(k_sweep_control, dim3(1), dim3(c.part ? PART_SLOTS : 1), 0, st, c);
}

hipError_t launch_global_relabel(int P, bool rc, int blocks, hipStream_t st, GRArgs &a) {
  void *args[] = {&a};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void *>(gr_fn(P, rc)), dim3(blocks), dim3(GR_THREADS), args,
                                    0, st);
}

int gr_max_blocks(int device, int P) {
  int per_cu = 1 << 30;
  for (int rc = 0; rc < 2; rc++) {  // both layouts' kernels must fit
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void *>(gr_fn(P, rc != 0)),
                                                      GR_THREADS, 0) != hipSuccess)
      return 0;
    per_cu = std::min(per_cu, n);
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  // one workgroup per CU: barrier latency grows with the number of
  // workgroups, and 16 waves per CU keep the BFS gathers in flight
  return std::min(per_cu, 1) * prop.multiProcessorCount;
}

}  // namespace wb
