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
//     a whole workgroup.
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
#include "wb_solver.h"

namespace wb {

struct Graph {
  int32_t V;
  int32_t hcap;
  const int32_t *rptr;
  int2 *ent;
  const int32_t *rev;
  long long *e;
  int32_t *h;
  int32_t sink;  // target of the current phase: its excess is never read, so
                 // pushes into it skip the excess atomic (-1: none skipped)
};

struct SweepQ {
  const int32_t *qin;
  const int32_t *qin_cnt;
  int32_t *qout;
  int32_t *qout_cnt;
  int32_t *zero_cnt;
  int32_t *mid_v;       // medium rows deferred to the one-wave tier
  int32_t *mid_cnt;
  int32_t *big_v;       // long rows deferred to the workgroup tier
  int32_t *big_cnt;
  int32_t *zero_a;      // counters to clear for the next sweep (nullable)
  int32_t *zero_b;
  int32_t t_mid;        // rows longer than this go to the one-wave tier
  int32_t t_big;        // rows longer than this go to the workgroup tier
  long long *stats;     // per kernel k (0 tile, 1 wave, 2 workgroup): [4k] arc scans, [4k+1] pushes,
                        // [4k+2] relabels, [4k+3] queued; [12] bfs scans; [13] nonempty sweeps
  int32_t qcap;      // capacity of every queue and of the long-row list (V)
  int32_t *err;      // overflow counter (must stay 0)
  int32_t mode;      // 0: one push to the minimum-height neighbour (Algorithms 1-2)
                     // 1: full discharge (push along every lower residual arc, then relabel)
};

// Pushes d along residual entry k of row u into v: the four atomic updates
// of Algorithm 1 except the decrement of e(u), which the caller applies once
// per visit.  Returns true when v's excess crossed from <= 0 to > 0 (v must
// then be enqueued, if it is not above the cap).
__device__ __forceinline__ bool push_entry(const Graph &g, int32_t k, int32_t v, long long d) {
  atomic_add_i32(&g.ent[k].y, -(int32_t)d);
  atomic_add_i32(&g.ent[g.rev[k]].y, (int32_t)d);
  if (v == g.sink) return false;
  long long oldv = atomic_add_i64(&g.e[v], d);
  return oldv <= 0 && oldv + d > 0;
}

__device__ __forceinline__ void flush_stats(long long *stats, long long scans, int pushes, int relabels, long long queued) {
  // one atomic per wave and counter
  scans = (long long)group_sum_i64<WB_WAVE>(scans);
  long long p = group_sum_i64<WB_WAVE>((long long)pushes);
  long long r = group_sum_i64<WB_WAVE>((long long)relabels);
  queued = group_sum_i64<WB_WAVE>(queued);
  if (lane() == 0) {
    if (scans) atomic_add_i64(&stats[0], scans);
    if (p) atomic_add_i64(&stats[1], p);
    if (r) atomic_add_i64(&stats[2], r);
    if (queued) atomic_add_i64(&stats[3], queued);
  }
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

constexpr int SWEEP_THREADS = 256;

// One visit of a queued vertex by a tile of P lanes (rows up to
// split_degree).  Paper mode: the tile reduces the packed key
// (height << 32 | row position) over residual entries to its minimum; the
// first lane pushes min(e(u), c_f) to that neighbour if it is lower, else
// relabels to its height + 1.  Discharge mode: the tile walks the row P
// entries at a time and pushes along every residual entry whose head is
// lower than u, handing out e(u) in row order with a prefix sum, stops once
// e(u) is spent, and relabels to 1 + the lowest remaining residual neighbour
// if excess is left.
template <int P>
__global__ void __launch_bounds__(SWEEP_THREADS) k_sweep_tile(Graph g, SweepQ q) {
  constexpr int DEFER_BUF = 128;
  __shared__ int s_qbuf[SWEEP_THREADS / WB_WAVE][WB_QBUF];
  __shared__ int s_mbuf[SWEEP_THREADS / WB_WAVE][DEFER_BUF];
  __shared__ int s_bbuf[SWEEP_THREADS / WB_WAVE][DEFER_BUF];
  __shared__ int s_qcnt[SWEEP_THREADS / WB_WAVE][3];
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
  if (blockIdx.x == 0 && threadIdx.x == 0 && q.zero_cnt) {
    *q.zero_cnt = 0;
    *q.zero_a = 0;
    *q.zero_b = 0;
    if (*q.qin_cnt > 0) atomic_add_i64(&q.stats[13], 1);
  }
  const int32_t n = min(*q.qin_cnt, q.qcap);
  constexpr int TPW = WB_WAVE / P;  // tiles per wave
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t wave = (int32_t)(gtid / WB_WAVE);
  const int32_t nwaves = (int32_t)((int64_t)gridDim.x * blockDim.x / WB_WAVE);
  const int sub = lane() / P;
  const int tl = lane() % P;
  const int tbase = lane() & ~(P - 1);
  long long scans = 0, queued = 0;
  int pushes = 0, relabels = 0;
  for (int32_t base = wave * TPW; base < n; base += nwaves * TPW) {  // wave-uniform loop
    const int32_t i = base + sub;
    const bool valid = i < n;
    int32_t u = 0, beg = 0, end = 0;
    if (valid) {
      u = q.qin[i];
      beg = g.rptr[u];
      end = g.rptr[u + 1];
    }
    const int32_t deg = end - beg;
    const bool split = valid && deg > q.t_mid;
    const bool scan = valid && !split;
    const bool leader = tl == 0;
    if (defers) {
      waveq_push(wmid, leader && split && deg <= q.t_big, u);
      waveq_push(wbig, leader && split && deg > q.t_big, u);
    }
    bool app_u = false;
    if (q.mode == 0) {
      unsigned long long key = WB_KEY_NONE;
      if (scan) {
        for (int32_t k = beg + tl; k < end; k += P) {
          int2 cr = g.ent[k];
          if (cr.y > 0) {
            unsigned long long kk = ((unsigned long long)(unsigned)g.h[cr.x] << 32) | (unsigned)(k - beg);
            key = kk < key ? kk : key;
          }
        }
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
            v = g.ent[k].x;
            long long eu = atomic_load_i64(&g.e[u]);
            long long d = eu < (long long)atomic_load_i32(&g.ent[k].y) ? eu : (long long)atomic_load_i32(&g.ent[k].y);
            if (d > 0) {
              app_v = push_entry(g, k, v, d) && g.h[v] < g.hcap;
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
            relabels++;
            app_u = nh < g.hcap;
          }
        }
      }
      waveq_push(wq, app_v, v);
    } else {
      // full discharge; every lane of a scanning tile iterates the same count
      const int32_t hu = scan ? g.h[u] : 0;
      long long e0 = (scan && leader) ? atomic_load_i64(&g.e[u]) : 0;
      e0 = (long long)shfl_u64((unsigned long long)e0, tbase);
      long long erem = e0;
      unsigned long long key = WB_KEY_NONE;  // lowest residual entry not lower than u
      long long nscan = 0;
      if (scan) {
        for (int32_t kb = beg; kb < end && erem > 0; kb += P) {
          const int32_t k = kb + tl;
          long long want = 0;
          int32_t v = 0;
          if (k < end) {
            int2 cr = g.ent[k];
            if (cr.y > 0) {
              const int32_t hv = g.h[cr.x];
              if (hv < hu) {
                want = cr.y;
                v = cr.x;
              } else {
                unsigned long long kk = ((unsigned long long)(unsigned)hv << 32) | (unsigned)(k - beg);
                key = kk < key ? kk : key;
              }
            }
          }
          long long tot;
          const long long before = group_excl_scan_i64<P>(want, &tot);
          long long take = erem - before;
          take = take < 0 ? 0 : (take > want ? want : take);
          bool app_v = false;
          if (take > 0) {
            app_v = push_entry(g, k, v, take) && g.h[v] < g.hcap;
            pushes++;
          }
          waveq_push(wq, app_v, v);
          erem -= tot;
          nscan += P;
        }
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
            relabels++;
            app_u = nh < g.hcap;
          }
        } else {
          app_u = left > 0;
        }
      }
    }
    waveq_push(wq, app_u, u);
  }
  waveq_flush(wq);
  if (defers) {
    waveq_flush(wmid);
    waveq_flush(wbig);
  }
  flush_stats(q.stats, scans, pushes, relabels, queued);
}

constexpr int BLK = 256;
constexpr int BLK_WAVES = BLK / WB_WAVE;

// Long rows: one workgroup per queued vertex, same two modes as the tile
// kernel with workgroup-wide reductions and prefix sums through LDS.
__global__ void __launch_bounds__(BLK) k_sweep_block(Graph g, SweepQ q) {
  __shared__ int s_qbuf[BLK_WAVES][WB_QBUF];
  __shared__ int s_qcnt[BLK_WAVES];
  __shared__ long long s_wsum[BLK_WAVES];
  __shared__ unsigned long long s_wmin[BLK_WAVES];
  __shared__ long long s_e0;
  const int32_t nbig = min(*q.big_cnt, q.qcap);
  const int w = threadIdx.x / WB_WAVE;
  if (lane() == 0) s_qcnt[w] = 0;
  const WaveQ wq{s_qbuf[w], &s_qcnt[w], q.qout, q.qout_cnt, q.qcap, q.err};
  long long scans = 0, queued = 0;
  int pushes = 0, relabels = 0;
  for (int32_t idx = blockIdx.x; idx < nbig; idx += gridDim.x) {
    const int32_t u = q.big_v[idx];
    const int32_t beg = g.rptr[u], end = g.rptr[u + 1];
    const int32_t hu = g.h[u];
    if (threadIdx.x == 0) s_e0 = atomic_load_i64(&g.e[u]);
    __syncthreads();
    const long long e0 = s_e0;
    long long erem = e0;
    unsigned long long key = WB_KEY_NONE;
    long long nscan = 0;
    for (int32_t kb = beg; kb < end && (q.mode == 0 || erem > 0); kb += BLK) {
      const int32_t k = kb + threadIdx.x;
      long long want = 0;
      int32_t v = 0;
      if (k < end) {
        int2 cr = g.ent[k];
        if (cr.y > 0) {
          const int32_t hv = g.h[cr.x];
          unsigned long long kk = ((unsigned long long)(unsigned)hv << 32) | (unsigned)(k - beg);
          if (q.mode == 1 && hv < hu) {
            want = cr.y;
            v = cr.x;
          } else {
            key = kk < key ? kk : key;
          }
        }
      }
      nscan += BLK;
      if (q.mode == 1) {
        long long wtot;
        long long before = group_excl_scan_i64<WB_WAVE>(want, &wtot);
        if (lane() == 0) s_wsum[w] = wtot;
        __syncthreads();
        long long off = 0, tot = 0;
#pragma unroll
        for (int j = 0; j < BLK_WAVES; j++) {
          long long x = s_wsum[j];
          off += j < w ? x : 0;
          tot += x;
        }
        __syncthreads();
        before += off;
        long long take = erem - before;
        take = take < 0 ? 0 : (take > want ? want : take);
        bool app_v = false;
        if (take > 0) {
          app_v = push_entry(g, k, v, take) && g.h[v] < g.hcap;
          pushes++;
        }
        waveq_push(wq, app_v, v);
        erem -= tot;
      }
    }
    key = group_min<WB_WAVE>(key);
    if (lane() == 0) s_wmin[w] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int j = 0; j < BLK_WAVES; j++) key = s_wmin[j] < key ? s_wmin[j] : key;
    }
    bool app_u = false, app_v = false;
    int32_t v = 0;
    if (threadIdx.x == 0) {
      scans += nscan < (end - beg) ? nscan : (end - beg);
      queued += 1;
      if (q.mode == 0) {
        if (key == WB_KEY_NONE) {
          app_u = true;
        } else {
          const int32_t hmin = (int32_t)(key >> 32);
          const int32_t k = beg + (int32_t)(key & 0xffffffffu);
          if (hu > hmin) {
            v = g.ent[k].x;
            const int32_t rk = atomic_load_i32(&g.ent[k].y);
            long long d = e0 < (long long)rk ? e0 : (long long)rk;
            if (d > 0) {
              app_v = push_entry(g, k, v, d) && g.h[v] < g.hcap;
              long long oldu = atomic_add_i64(&g.e[u], -d);
              app_u = oldu - d > 0;
              pushes++;
            } else {
              app_u = e0 > 0;
            }
          } else {
            int32_t nh = hmin + 1;
            if (nh > g.hcap) nh = g.hcap;
            g.h[u] = nh;
            relabels++;
            app_u = nh < g.hcap;
          }
        }
      } else {
        const long long pushed = e0 - (erem > 0 ? erem : 0);
        long long left = e0;
        if (pushed > 0) left = atomic_add_i64(&g.e[u], -pushed) - pushed;
        if (erem > 0) {
          if (key == WB_KEY_NONE) {
            app_u = true;
          } else {
            int32_t nh = (int32_t)(key >> 32) + 1;
            if (nh > g.hcap) nh = g.hcap;
            g.h[u] = nh;
            relabels++;
            app_u = nh < g.hcap;
          }
        } else {
          app_u = left > 0;
        }
      }
    }
    if (w == 0) {
      waveq_push(wq, app_v, v);
      waveq_push(wq, app_u, u);
    }
    __syncthreads();
  }
  waveq_flush(wq);
  flush_stats(q.stats + 8, scans, pushes, relabels, queued);
}

// ------------------------------------------------------ global relabel
struct GRArgs {
  Graph g;
  int32_t root, excl, root_h;
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
  long long *stats;
  long long *status;  // [0] active, [1] stranded, [2] levels, [3] bottom-up levels
  int32_t split_deg, chunk;
  int32_t qcap;       // capacity of frontiers and queue (V)
  int32_t chunk_cap;  // capacity of the chunk descriptor arrays
  int32_t bu_threshold;    // frontier size above which a level runs bottom-up
  long long bu_edges;      // frontier row-length sum above which a level runs bottom-up
  int32_t *err;       // overflow counter (must stay 0)
};

__device__ __forceinline__ uint8_t dist_code(int32_t d) { return (uint8_t)(1 + (d & 1)); }

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
constexpr int GR_THREADS = 1024;

template <int P>
__global__ void __launch_bounds__(GR_THREADS) k_global_relabel(GRArgs a) {
  __shared__ int s_qbuf[GR_THREADS / WB_WAVE][WB_QBUF];
  __shared__ int s_qcnt[GR_THREADS / WB_WAVE];
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

  for (int64_t v = gtid; v < g.V; v += nthreads) {
    g.h[v] = g.hcap;
    a.vis[v] = 0;
  }
  if (gtid == 0) {
    a.fcnt[0] = 1;
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
    a.fq[0][0] = a.root;
  }
  grid_barrier(a.bar, nblocks);
  if (gtid == 0) {
    g.h[a.root] = a.root_h;
    a.vis[a.root] = dist_code(0);
    if (a.excl >= 0) {
      g.h[a.excl] = g.hcap + 1;
      a.vis[a.excl] = 3;
    }
  }
  grid_barrier(a.bar, nblocks);

  long long bscans = 0, buscans = 0;  // entries examined top-down / bottom-up
  int32_t level = 0, bu_levels = 0;
  int32_t n = 1;
  long long nedges = 0;  // row-length sum of the current frontier (0: the root alone)
  bool queue_valid = true;  // the frontier of this level is in fq[level & 1]
  for (;;) {
    if (n == 0) break;
    const uint8_t cur = dist_code(level), nxt = dist_code(level + 1);
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
    const bool bottom_up = n > a.bu_threshold || nedges > a.bu_edges;
    if (bottom_up) {
      bu_levels++;
      // every unvisited vertex with a short row: tile of P lanes, stop at
      // the first residual arc into the frontier; long rows become chunks
      int found_cnt = 0;
      int32_t *ccnt = &a.chunk_cnt[level & 1];
      for (int64_t vb = (int64_t)wave * TPW; vb < g.V; vb += (int64_t)nwaves * TPW) {
        const int64_t v = vb + sub;
        bool mine = v < g.V && a.vis[v] == 0;
        int32_t beg = 0, end = 0;
        if (mine) {
          beg = g.rptr[v];
          end = g.rptr[v + 1];
        }
        if (mine && end - beg > a.split_deg) {
          mine = false;
          if (tl == 0) {
            const int32_t nch = (end - beg + a.chunk - 1) / a.chunk;
            const int32_t c0 = atomic_add_i32(ccnt, nch);
            if (c0 + nch <= a.chunk_cap) {
              for (int32_t j = 0; j < nch; j++) {
                a.chunk_w[c0 + j] = (int32_t)v;
                a.chunk_b[c0 + j] = beg + j * a.chunk;
              }
            } else {
              atomic_add_i32(a.err, 1);
            }
          }
        }
        if (mine) {
          for (int32_t kb = beg; kb < end; kb += P) {  // tile-uniform trip count
            const int32_t k = kb + tl;
            bool hit = false;
            int32_t w = 0;
            if (k < end) {
              const int2 cr = g.ent[k];
              w = cr.x;
              hit = cr.y > 0 && a.vis[w] == cur;
            }
            const unsigned long long m = (__ballot(hit) >> tbase) & (P == 64 ? ~0ull : ((1ull << P) - 1));
            if (tl == 0) buscans += min(P, end - kb);
            if (m) {
              if (tl == __ffsll((long long)m) - 1) {
                g.h[v] = g.h[w] + 1;
                a.vis[v] = nxt;
                found_cnt++;
                my_edges += end - beg;
              }
              break;
            }
          }
        }
      }
      // publish this phase's counts before the barrier
      found_cnt = wave_sum_i32(found_cnt);
      my_edges = group_sum_i64<WB_WAVE>(my_edges);
      if (lane() == 0 && found_cnt) atomic_add_i32(&a.bucnt[(level + 1) % 3], found_cnt);
      if (lane() == 0 && my_edges) atomic_add_i64(fe_out, my_edges);
      found_cnt = 0;
      my_edges = 0;
      grid_barrier(a.bar, nblocks);
      // long unvisited rows: one wave per chunk; a hit claims v by CAS.
      // nc is read after the barrier, so every workgroup agrees on it and on
      // whether the second barrier below is needed.
      const int32_t nc = min(atomic_load_i32(ccnt), a.chunk_cap);
      for (int32_t c = wave; c < nc; c += nwaves) {
        const int32_t v = a.chunk_w[c];
        const int32_t cb = a.chunk_b[c];
        const int32_t ce = min(cb + a.chunk, g.rptr[v + 1]);
        if (lane() == 0) buscans += ce - cb;
        for (int32_t kb = cb; kb < ce; kb += WB_WAVE) {
          const int32_t k = kb + lane();
          bool hit = false;
          int32_t w = 0;
          if (k < ce) {
            const int2 cr = g.ent[k];
            w = cr.x;
            hit = cr.y > 0 && a.vis[w] == cur;
          }
          const unsigned long long m = __ballot(hit);
          if (m) {
            if (lane() == __ffsll((long long)m) - 1) {
              if (atomicCAS(&g.h[v], g.hcap, g.h[w] + 1) == g.hcap) {
                a.vis[v] = nxt;
                found_cnt++;
                my_edges += g.rptr[v + 1] - g.rptr[v];
              }
            }
            break;
          }
        }
      }
      if (nc > 0) {
        found_cnt = wave_sum_i32(found_cnt);
        my_edges = group_sum_i64<WB_WAVE>(my_edges);
        if (lane() == 0 && found_cnt) atomic_add_i32(&a.bucnt[(level + 1) % 3], found_cnt);
        if (lane() == 0 && my_edges) atomic_add_i64(fe_out, my_edges);
        grid_barrier(a.bar, nblocks);
      }
      n = min(atomic_load_i32(&a.bucnt[(level + 1) % 3]), a.qcap);
      nedges = atomic_load_i64(fe_out);
      queue_valid = false;
    } else {
      const int32_t *fin = a.fq[level & 1];
      if (!queue_valid) {
        // the frontier was produced bottom-up: list the vertices of code(L)
        WaveQ wq{s_qbuf[wl], &s_qcnt[wl], a.fq[level & 1], &a.fcnt[level % 3], a.qcap, a.err};
        if (gtid == 0) a.fcnt[level % 3] = 0;
        grid_barrier(a.bar, nblocks);
        for (int64_t v0 = gtid - lane(); v0 < g.V; v0 += nthreads) {
          const int64_t v = v0 + lane();
          waveq_push(wq, v < g.V && a.vis[v] == cur, (int32_t)v);
        }
        waveq_flush(wq);
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
          const int32_t beg = g.rptr[w], end = g.rptr[w + 1];
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
              const int32_t v = g.ent[k].x;
              bool claimed = false;
              if (g.h[v] == g.hcap && g.ent[g.rev[k]].y > 0) {
                claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
                if (claimed) {
                  a.vis[v] = nxt;
                  my_edges += g.rptr[v + 1] - g.rptr[v];
                }
              }
              waveq_push(wq, claimed, v);
            }
          }
        }
      }
      waveq_flush(wq);
      my_edges = group_sum_i64<WB_WAVE>(my_edges);
      if (lane() == 0 && my_edges) atomic_add_i64(fe_out, my_edges);
      my_edges = 0;
      grid_barrier(a.bar, nblocks);
      // phase B: one wave per chunk of a long row (skipped, with its barrier,
      // when the level met no long row: nc is read after the barrier)
      const int32_t nc = min(atomic_load_i32(ccnt), a.chunk_cap);
      for (int32_t c = wave; c < nc; c += nwaves) {
        const int32_t w = a.chunk_w[c];
        const int32_t cb = a.chunk_b[c];
        const int32_t ce = min(cb + a.chunk, g.rptr[w + 1]);
        const int32_t hw1 = g.h[w] + 1;
        if (lane() == 0) bscans += ce - cb;
        for (int32_t k = cb + lane(); k < ce; k += WB_WAVE) {
          const int32_t v = g.ent[k].x;
          bool claimed = false;
          if (g.h[v] == g.hcap && g.ent[g.rev[k]].y > 0) {
            claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
            if (claimed) {
              a.vis[v] = nxt;
              my_edges += g.rptr[v + 1] - g.rptr[v];
            }
          }
          waveq_push(wq, claimed, v);
        }
      }
      if (nc > 0) {
        waveq_flush(wq);
        my_edges = group_sum_i64<WB_WAVE>(my_edges);
        if (lane() == 0 && my_edges) atomic_add_i64(fe_out, my_edges);
        grid_barrier(a.bar, nblocks);
      }
      n = min(atomic_load_i32(fout_cnt), a.qcap);
      nedges = atomic_load_i64(fe_out);
      queue_valid = true;
    }
    level++;
  }
  // rebuild the active-vertex queue; count excess stranded away from the root
  int stranded = 0;
  {
    WaveQ wq{s_qbuf[wl], &s_qcnt[wl], a.qout, &a.qcnt[0], a.qcap, a.err};
    for (int64_t v0 = gtid - lane(); v0 < g.V; v0 += nthreads) {  // wave-uniform
      const int64_t v = v0 + lane();
      bool act = false;
      if (v < g.V) {
        const long long ev = g.e[v];
        const int32_t hv = g.h[v];
        act = ev > 0 && hv < g.hcap;
        stranded += (ev > 0 && hv == g.hcap) ? 1 : 0;
      }
      waveq_push(wq, act, (int32_t)v);
    }
    waveq_flush(wq);
  }
  stranded = wave_sum_i32(stranded);
  const long long bs = group_sum_i64<WB_WAVE>(bscans);
  const long long bus = group_sum_i64<WB_WAVE>(buscans);
  if (lane() == 0) {
    if (stranded) atomic_add_i64(&a.status[1], stranded);
    if (bs) atomic_add_i64(&a.stats[12], bs);
    if (bus) atomic_add_i64(&a.stats[14], bus);
  }
  grid_barrier(a.bar, nblocks);
  if (gtid == 0) {
    a.status[0] = a.qcnt[0];
    a.status[2] = level;
    a.status[3] = bu_levels;
  }
}

// ------------------------------------------------------------ small kernels
__global__ void k_init(Graph g, int32_t t) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.V; v += (int64_t)gridDim.x * blockDim.x) {
    g.e[v] = (v == t) ? WB_EXCESS_BIAS : 0;
    g.h[v] = 0;
  }
}

// Preflow (Algorithm 1, step 0): every residual entry of s is saturated.
__global__ void k_preflow(Graph g, int32_t s) {
  const int32_t beg = g.rptr[s], end = g.rptr[s + 1];
  for (int64_t k = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < end;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int2 cr = g.ent[k];
    if (cr.y > 0) {
      g.ent[k].y = 0;
      atomic_add_i32(&g.ent[g.rev[k]].y, cr.y);
      atomic_add_i64(&g.e[cr.x], (long long)cr.y);
    }
  }
}

__global__ void k_add_excess(long long *e, int32_t v, long long d) { e[v] += d; }

__global__ void k_zero_i64(long long *out) { out[0] = 0; }

// Flow value = total flow into t = sum over t's row of (c_f(t,w) - c(t,w)):
// every push w -> t raised the mate residual c_f(t,w) by the pushed amount
// and nothing ever pushes out of t, so t's excess need not be tracked.
__global__ void k_value(Graph g, const int32_t *cap0, int32_t t, long long *out) {
  __shared__ long long s_part[SWEEP_THREADS / WB_WAVE];
  const int32_t beg = g.rptr[t], end = g.rptr[t + 1];
  long long acc = 0;
  for (int64_t k = beg + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < end;
       k += (int64_t)gridDim.x * blockDim.x)
    acc += (long long)g.ent[k].y - (long long)cap0[k];
  acc = group_sum_i64<WB_WAVE>(acc);
  if (lane() == 0) s_part[threadIdx.x / WB_WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long tot = 0;
    for (int i = 0; i < SWEEP_THREADS / WB_WAVE; i++) tot += s_part[i];
    if (tot) atomic_add_i64(out, tot);
  }
}

__global__ void k_cut_side(Graph g, uint8_t *side) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.V; v += (int64_t)gridDim.x * blockDim.x)
    side[v] = g.h[v] < g.hcap ? 1 : 0;
}

// Per-arc flow from the merged net flow of the ordered pair (u,v): parallel
// arcs u->v are filled in input order up to their capacities.
__global__ void k_decode(int64_t E, const int32_t *cap, const int32_t *arc2ent, const int32_t *pbefore,
                         const int32_t *cap0, const int2 *ent, int32_t *flow) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = arc2ent[i];
    int32_t f = 0;
    if (j >= 0) {
      const long long net = (long long)cap0[j] - (long long)ent[j].y;
      long long x = net - (long long)pbefore[i];
      if (x < 0) x = 0;
      if (x > cap[i]) x = cap[i];
      f = (int32_t)x;
    }
    flow[i] = f;
  }
}

// ------------------------------------------------------------ host driver
// WBPR_LOG=1 traces every global-relabel round on stderr.
static int log_level() {
  static int lvl = -1;
  if (lvl < 0) {
    const char *e = std::getenv("WBPR_LOG");
    lvl = e ? std::atoi(e) : 0;
  }
  return lvl;
}

static unsigned grid1d(int64_t n, int threads = 256, int64_t maxb = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > maxb) b = maxb;
  return (unsigned)b;
}

typedef void (*TileFn)(Graph, SweepQ);
typedef void (*GRFn)(GRArgs);

static TileFn tile_fn(int P) {
  switch (P) {
    case 4: return k_sweep_tile<4>;
    case 8: return k_sweep_tile<8>;
    case 16: return k_sweep_tile<16>;
    case 32: return k_sweep_tile<32>;
    default: return k_sweep_tile<64>;
  }
}
static GRFn gr_fn(int P) {
  switch (P) {
    case 4: return k_global_relabel<4>;
    case 8: return k_global_relabel<8>;
    case 16: return k_global_relabel<16>;
    case 32: return k_global_relabel<32>;
    default: return k_global_relabel<64>;
  }
}

int gr_max_blocks(int device, int P) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(gr_fn(P)), GR_THREADS,
                                                    0) != hipSuccess)
    return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  // one workgroup per CU: barrier latency grows with the number of
  // workgroups, and 16 waves per CU keep the BFS gathers in flight
  return std::min(per_cu, 1) * prop.multiProcessorCount;
}

// Long rows met in one BFS level produce at most M/chunk + (number of long
// rows) <= M/chunk + V chunk descriptors.
static int64_t chunk_capacity(int32_t V, int64_t Mcap, int chunk) { return Mcap / chunk + V + 16; }

size_t state_bytes(int32_t V, int64_t Mcap, int chunk) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  int64_t nchunk = chunk_capacity(V, Mcap, chunk);
  return al(8ull * V) + al(4ull * V) * 7 + al((size_t)V) + al(4ull * nchunk) * 2 + al(4096);
}

void state_carve(State *s, int32_t V, int64_t Mcap, int chunk, void *mem) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char *p = (char *)mem;
  int64_t nchunk = chunk_capacity(V, Mcap, chunk);
  s->e = (long long *)p; p += al(8ull * V);
  s->h = (int32_t *)p; p += al(4ull * V);
  s->q[0] = (int32_t *)p; p += al(4ull * V);
  s->q[1] = (int32_t *)p; p += al(4ull * V);
  s->fq[0] = (int32_t *)p; p += al(4ull * V);
  s->fq[1] = (int32_t *)p; p += al(4ull * V);
  s->big_v = (int32_t *)p; p += al(4ull * V);
  s->mid_v = (int32_t *)p; p += al(4ull * V);
  s->vis = (uint8_t *)p; p += al((size_t)V);
  s->chunk_w = (int32_t *)p; p += al(4ull * nchunk);
  s->chunk_b = (int32_t *)p; p += al(4ull * nchunk);
  s->misc = (long long *)p;  // 4 KB of counters
  s->nchunk_cap = nchunk;
}

namespace {
struct MiscLayout {
  long long stats[16];
  long long status[4];
  int32_t err[2];
  int32_t big_cnt[2];
  int32_t mid_cnt[2];
  int32_t bucnt[4];
  int32_t qcnt[4];
  int32_t fcnt[4];
  int32_t chunk_cnt[2];
  unsigned bar[WB_BAR_WORDS];
  long long fedges[4];
};
}  // namespace

size_t misc_bytes() { return sizeof(MiscLayout); }

static int pick_lanes(const SolveConfig &cfg, int32_t V, int64_t M) {
  if (cfg.lanes_per_vertex) return cfg.lanes_per_vertex;
  double avg = V > 0 ? (double)M / (double)V : 1.0;
  int P = 4;
  while (P < 64 && P < avg) P <<= 1;
  return P;
}

// Runs one phase (sink = root) to completion.  Returns 0 or a wbpr status.
struct Tiers {
  int P;           // lanes per short row
  int32_t t_mid;   // rows longer than this: one wave each
  int32_t t_big;   // rows longer than this: one workgroup each
  int32_t bfs_split, chunk;
};

static int run_phase(const SolveConfig &cfg, const Residual &res, State &S, int32_t root, int32_t excl,
                     const Tiers &tiers, int gr_blocks, hipStream_t st, long long *pinned, PhaseStats *ps,
                     bool second_phase, std::string *err) {
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(S.misc);
  Graph g{res.V, res.V, res.rptr, res.ent, res.rev, S.e, S.h, root};
  GRArgs ga;
  ga.g = g;
  ga.root = root;
  ga.excl = excl;
  ga.root_h = 0;
  ga.fq[0] = S.fq[0];
  ga.fq[1] = S.fq[1];
  ga.fcnt = misc->fcnt;
  ga.chunk_w = S.chunk_w;
  ga.chunk_b = S.chunk_b;
  ga.chunk_cnt = misc->chunk_cnt;
  ga.bar = misc->bar;
  ga.qout = S.q[0];
  ga.qcnt = misc->qcnt;
  ga.big_cnt = misc->big_cnt;
  ga.stats = misc->stats;
  ga.status = misc->status;
  ga.split_deg = tiers.bfs_split;
  ga.chunk = tiers.chunk;
  ga.vis = S.vis;
  ga.bucnt = misc->bucnt;
  ga.bu_threshold = std::max<int32_t>(res.V / 32, 4096);
  ga.bu_edges = std::max<long long>(res.M / 16, 65536);
  ga.fedges = misc->fedges;
  ga.qcap = res.V;
  ga.chunk_cap = (int32_t)std::min<int64_t>(S.nchunk_cap, 0x7fffffff);
  ga.err = misc->err;
  TileFn tfn = tile_fn(tiers.P);
  TileFn wfn = tile_fn(64);
  GRFn gfn = gr_fn(tiers.P);
  const int K = cfg.gr_every_sweeps > 0 ? cfg.gr_every_sweeps : 16;
  const int sweep_blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : 1024;
  const int block_blocks = 512;
  const int mode = cfg.push_mode == 1 ? 0 : 1;
  auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipError_t he = hipMemsetAsync(misc->status, 0, sizeof(misc->status), st);
    if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
    void *args[] = {&ga};
    auto tg0 = std::chrono::steady_clock::now();
    const bool time_gr = cfg.time_kernels && S.gev_count < State::kMaxGR;
    if (time_gr) hipEventRecord(S.gev[S.gev_count][0], st);
    he = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(gfn), dim3(gr_blocks), dim3(GR_THREADS), args, 0,
                                    st);
    if (he != hipSuccess) { *err = std::string("global relabel launch: ") + hipGetErrorString(he); return 5; }
    if (time_gr) hipEventRecord(S.gev[S.gev_count++][1], st);
    ps->global_relabels++;
    he = hipMemcpyAsync(pinned, misc->status, sizeof(misc->status) + sizeof(misc->err), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) { *err = std::string("global relabel: ") + hipGetErrorString(he); return 5; }
    const long long active = pinned[0];
    const long long stranded = pinned[1];
    ps->gr_levels += pinned[2];
    if (log_level() > 0) {
      double gms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg0).count();
      std::fprintf(stderr,
                   "[wbpr] phase %d round %lld: active=%lld stranded=%lld bfs_levels=%lld (bottom-up %lld) "
                   "gr+sync=%.3f ms sweeps so far=%lld\n",
                   second_phase ? 2 : 1, (long long)ps->global_relabels, active, stranded, pinned[2], pinned[3], gms,
                   (long long)ps->sweeps);
    }
    const int32_t *errw = reinterpret_cast<const int32_t *>(&pinned[4]);
    if (errw[0] != 0) {
      *err = "internal queue overflow";
      return 8;
    }
    if (second_phase && stranded > 0) {
      *err = "second phase: excess that cannot return to the source";
      return 8;
    }
    if (active == 0) break;
    if (cfg.max_sweeps > 0 && ps->sweeps >= cfg.max_sweeps) { *err = "max_sweeps exceeded"; return 4; }
    if (cfg.max_wall_ms > 0) {
      double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      if (ms > cfg.max_wall_ms) { *err = "max_wall_ms exceeded"; return 4; }
    }
    for (int j = 0; j < K; j++) {
      // short rows: tiles of P lanes; medium and long rows are deferred
      SweepQ q;
      q.qin = S.q[j & 1];
      q.qin_cnt = &misc->qcnt[j % 3];
      q.qout = S.q[(j + 1) & 1];
      q.qout_cnt = &misc->qcnt[(j + 1) % 3];
      q.zero_cnt = &misc->qcnt[(j + 2) % 3];
      q.mid_v = S.mid_v;
      q.mid_cnt = &misc->mid_cnt[j & 1];
      q.big_v = S.big_v;
      q.big_cnt = &misc->big_cnt[j & 1];
      q.zero_a = &misc->mid_cnt[(j + 1) & 1];
      q.zero_b = &misc->big_cnt[(j + 1) & 1];
      q.t_mid = tiers.t_mid;
      q.t_big = tiers.t_big;
      q.mode = mode;
      q.stats = misc->stats;
      q.qcap = res.V;
      q.err = misc->err;
      // medium rows: one wave each, nothing deferred further
      SweepQ qw = q;
      qw.qin = S.mid_v;
      qw.qin_cnt = &misc->mid_cnt[j & 1];
      qw.zero_cnt = nullptr;
      qw.t_mid = 0x7fffffff;
      qw.t_big = 0x7fffffff;
      qw.stats = misc->stats + 4;
      const bool timed = cfg.time_kernels && S.ev_count < State::kMaxSweeps;
      hipEvent_t *ev = timed ? S.ev[S.ev_count++] : nullptr;
      if (timed) hipEventRecord(ev[0], st);
      hipLaunchKernelGGL(tfn, dim3(sweep_blocks), dim3(SWEEP_THREADS), 0, st, g, q);
      if (timed) hipEventRecord(ev[1], st);
      hipLaunchKernelGGL(wfn, dim3(sweep_blocks), dim3(SWEEP_THREADS), 0, st, g, qw);
      if (timed) hipEventRecord(ev[2], st);
      hipLaunchKernelGGL(k_sweep_block, dim3(block_blocks), dim3(BLK), 0, st, g, q);
      if (timed) hipEventRecord(ev[3], st);
      ps->sweeps++;
    }
    he = hipGetLastError();
    if (he != hipSuccess) { *err = std::string("sweep launch: ") + hipGetErrorString(he); return 5; }
  }
  return 0;
}

int solve_on_device(const SolveConfig &cfg, const Residual &res, State &S, int32_t s, int32_t t, const int *gr_blocks_tab,
                    hipStream_t st, long long *pinned, int64_t *dev_value, int32_t *dev_flow, uint8_t *dev_side,
                    const int32_t *dev_cap, SolveReport *rep, std::string *err) {
  Tiers tiers;
  tiers.P = cfg.lanes_per_vertex > 0 ? cfg.lanes_per_vertex : 8;
  tiers.t_mid = cfg.split_degree > 0 ? cfg.split_degree : 4 * tiers.P;
  tiers.t_big = cfg.block_degree > 0 ? cfg.block_degree : std::max<int32_t>(tiers.t_mid, 2048);
  if (tiers.t_big < tiers.t_mid) tiers.t_big = tiers.t_mid;
  tiers.bfs_split = 8 * tiers.P;
  tiers.chunk = 1024;
  int lg = 0;
  while ((1 << lg) < tiers.P) lg++;
  const int gr_blocks = std::min(gr_blocks_tab[lg], 1024);
  if (gr_blocks < 1) { *err = "cooperative launch not possible"; return 5; }
  rep->lanes = tiers.P;
  rep->split_degree = tiers.t_mid;
  rep->block_degree = tiers.t_big;
  rep->gr_blocks = gr_blocks;
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(S.misc);
  Graph g{res.V, res.V, res.rptr, res.ent, res.rev, S.e, S.h, -1};
  hipMemsetAsync(S.misc, 0, sizeof(MiscLayout), st);
  hipLaunchKernelGGL(k_init, dim3(grid1d(res.V)), dim3(256), 0, st, g, t);
  hipLaunchKernelGGL(k_preflow, dim3(grid1d(res.M > 0 ? res.M : 1, 256, 4096)), dim3(256), 0, st, g, s);
  auto t0 = std::chrono::steady_clock::now();
  PhaseStats p1{}, p2{};
  int rc = run_phase(cfg, res, S, t, s, tiers, gr_blocks, st, pinned, &p1, false, err);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, st, (long long *)dev_value);
  hipLaunchKernelGGL(k_value, dim3(256), dim3(SWEEP_THREADS), 0, st, g, res.cap0, t, (long long *)dev_value);
  if (dev_side) hipLaunchKernelGGL(k_cut_side, dim3(grid1d(res.V)), dim3(256), 0, st, g, dev_side);
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
  auto t1 = std::chrono::steady_clock::now();
  if (dev_flow) {
    // second phase: return the excess stranded in the source side to s
    hipLaunchKernelGGL(k_add_excess, dim3(1), dim3(1), 0, st, S.e, s, (long long)WB_EXCESS_BIAS);
    rc = run_phase(cfg, res, S, s, t, tiers, gr_blocks, st, pinned, &p2, true, err);
    if (rc) return rc;
    auto t2 = std::chrono::steady_clock::now();
    hipLaunchKernelGGL(k_decode, dim3(grid1d(res.E > 0 ? res.E : 1)), dim3(256), 0, st, res.E, dev_cap, res.arc2ent,
                       res.pbefore, res.cap0, res.ent, dev_flow);
    he = hipStreamSynchronize(st);
    if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
    auto t3 = std::chrono::steady_clock::now();
    rep->ms_phase2 = std::chrono::duration<double, std::milli>(t2 - t1).count();
    rep->ms_decode = std::chrono::duration<double, std::milli>(t3 - t2).count();
  }
  rep->ms_phase1 = std::chrono::duration<double, std::milli>(t1 - t0).count();
  he = hipMemcpyAsync(pinned, misc->stats, sizeof(misc->stats), hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
  for (int k = 0; k < 3; k++) {
    rep->k_scans[k] = pinned[4 * k + 0];
    rep->k_pushes[k] = pinned[4 * k + 1];
    rep->k_relabels[k] = pinned[4 * k + 2];
    rep->k_queued[k] = pinned[4 * k + 3];
    rep->arc_scans += rep->k_scans[k];
    rep->pushes += rep->k_pushes[k];
    rep->relabels += rep->k_relabels[k];
    rep->queued += rep->k_queued[k];
  }
  rep->k_scans[3] = pinned[12] + pinned[14];
  rep->bfs_topdown_scans = pinned[12];
  rep->bfs_scans = pinned[12] + pinned[14];
  rep->nonempty_sweeps = pinned[13];
  rep->sweeps = p1.sweeps + p2.sweeps;
  rep->phase2_sweeps = p2.sweeps;
  rep->global_relabels = p1.global_relabels + p2.global_relabels;
  rep->gr_levels = p1.gr_levels + p2.gr_levels;
  if (cfg.time_kernels) {
    for (int i = 0; i < S.ev_count; i++) {
      for (int k = 0; k < 3; k++) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, S.ev[i][k], S.ev[i][k + 1]) == hipSuccess) rep->k_ms[k] += ms;
      }
    }
    for (int i = 0; i < S.gev_count; i++) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, S.gev[i][0], S.gev[i][1]) == hipSuccess) rep->k_ms[3] += ms;
    }
    rep->k_launches[0] = rep->k_launches[1] = rep->k_launches[2] = S.ev_count;
    rep->k_launches[3] = S.gev_count;
  }
  return 0;
}

}  // namespace wb
