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
};

struct SweepQ {
  const int32_t *qin;
  const int32_t *qin_cnt;
  int32_t *qout;
  int32_t *qout_cnt;
  int32_t *zero_cnt;
  int32_t *big_v;       // long rows deferred to the workgroup kernel
  int32_t *big_cnt;
  int32_t *big_cnt_zero;
  long long *stats;  // tile kernel [0] arc scans [1] pushes [2] relabels [3] queued; [4] bfs scans;
                     // [5] nonempty sweeps; workgroup kernel [8] arc scans [9] pushes [10] relabels [11] queued
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
__global__ void __launch_bounds__(SWEEP_THREADS) k_sweep_tile(Graph g, SweepQ q, int32_t split_deg) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *q.zero_cnt = 0;
    *q.big_cnt_zero = 0;
    if (*q.qin_cnt > 0) atomic_add_i64(&q.stats[5], 1);
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
    const bool split = valid && deg > split_deg;
    const bool scan = valid && !split;
    const bool leader = tl == 0;
    if (leader && split) {
      int32_t slot = atomic_add_i32(q.big_cnt, 1);
      if (slot < q.qcap) q.big_v[slot] = u;
      else atomic_add_i32(q.err, 1);
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
      wave_append(app_v, v, q.qout, q.qout_cnt, q.qcap, q.err);
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
          wave_append(app_v, v, q.qout, q.qout_cnt, q.qcap, q.err);
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
    wave_append(app_u, u, q.qout, q.qout_cnt, q.qcap, q.err);
  }
  flush_stats(q.stats, scans, pushes, relabels, queued);
}

constexpr int BLK = 256;
constexpr int BLK_WAVES = BLK / WB_WAVE;

// Long rows: one workgroup per queued vertex, same two modes as the tile
// kernel with workgroup-wide reductions and prefix sums through LDS.
__global__ void __launch_bounds__(BLK) k_sweep_block(Graph g, SweepQ q) {
  __shared__ long long s_wsum[BLK_WAVES];
  __shared__ unsigned long long s_wmin[BLK_WAVES];
  __shared__ long long s_e0;
  const int32_t nbig = min(*q.big_cnt, q.qcap);
  const int w = threadIdx.x / WB_WAVE;
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
        wave_append(app_v, v, q.qout, q.qout_cnt, q.qcap, q.err);
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
      wave_append(app_v, v, q.qout, q.qout_cnt, q.qcap, q.err);
      wave_append(app_u, u, q.qout, q.qout_cnt, q.qcap, q.err);
    }
    __syncthreads();
  }
  flush_stats(q.stats + 8, scans, pushes, relabels, queued);
}

// ------------------------------------------------------ global relabel
struct GRArgs {
  Graph g;
  int32_t root, excl, root_h;
  int32_t *fq[2];
  int32_t *fcnt;      // [3] rotating frontier counters
  int32_t *chunk_w;   // split rows: vertex
  int32_t *chunk_b;   //             first entry of the chunk
  int32_t *chunk_cnt; // [2]
  unsigned *bar;      // [2] barrier state
  int32_t *qout;      // active-vertex queue rebuilt at the end
  int32_t *qcnt;      // [3] sweep counters: [0] = queue length, [1],[2] zeroed
  int32_t *big_cnt;   // [2] zeroed
  long long *stats;
  long long *status;  // [0] active, [1] stranded, [2] levels
  int32_t split_deg, chunk;
  int32_t qcap;       // capacity of frontiers and queue (V)
  int32_t chunk_cap;  // capacity of the chunk descriptor arrays
  int32_t *err;       // overflow counter (must stay 0)
};

template <int P>
__global__ void __launch_bounds__(SWEEP_THREADS) k_global_relabel(GRArgs a) {
  const Graph &g = a.g;
  const unsigned nblocks = gridDim.x;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int32_t wave = (int32_t)(gtid / WB_WAVE);
  const int32_t nwaves = (int32_t)(nthreads / WB_WAVE);
  constexpr int TPW = WB_WAVE / P;
  const int sub = lane() / P;
  const int tl = lane() % P;

  for (int64_t v = gtid; v < g.V; v += nthreads) g.h[v] = g.hcap;
  if (gtid == 0) {
    a.fcnt[0] = 1;
    a.fcnt[1] = 0;
    a.fcnt[2] = 0;
    a.chunk_cnt[0] = 0;
    a.chunk_cnt[1] = 0;
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
    if (a.excl >= 0) g.h[a.excl] = g.hcap + 1;
  }
  grid_barrier(a.bar, nblocks);

  long long bscans = 0;
  int32_t level = 0;
  for (;;) {
    const int32_t n = min(atomic_load_i32(&a.fcnt[level % 3]), a.qcap);
    if (n == 0) break;
    const int32_t *fin = a.fq[level & 1];
    int32_t *fout = a.fq[(level + 1) & 1];
    int32_t *fout_cnt = &a.fcnt[(level + 1) % 3];
    int32_t *ccnt = &a.chunk_cnt[level & 1];
    if (gtid == 0) {
      a.fcnt[(level + 2) % 3] = 0;
      a.chunk_cnt[(level + 1) & 1] = 0;
    }
    // phase A: tiles of P lanes expand short rows, long rows become chunks
    for (int32_t base = wave * TPW; base < n; base += nwaves * TPW) {
      const int32_t i = base + sub;
      if (i < n) {
        const int32_t w = fin[i];
        const int32_t beg = g.rptr[w], end = g.rptr[w + 1];
        const int32_t deg = end - beg;
        if (deg > a.split_deg) {
          if (tl == 0) {
            int32_t nch = (deg + a.chunk - 1) / a.chunk;
            int32_t c0 = atomic_add_i32(ccnt, nch);
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
            if (g.h[v] == g.hcap && g.ent[g.rev[k]].y > 0) claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
            wave_append(claimed, v, fout, fout_cnt, a.qcap, a.err);
          }
        }
      }
    }
    grid_barrier(a.bar, nblocks);
    // phase B: one wave per chunk of a long row
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
        if (g.h[v] == g.hcap && g.ent[g.rev[k]].y > 0) claimed = atomicCAS(&g.h[v], g.hcap, hw1) == g.hcap;
        wave_append(claimed, v, fout, fout_cnt, a.qcap, a.err);
      }
    }
    grid_barrier(a.bar, nblocks);
    level++;
  }
  // rebuild the active-vertex queue; count excess stranded away from the root
  int stranded = 0;
  for (int64_t v0 = gtid - lane(); v0 < g.V; v0 += nthreads) {  // wave-uniform
    const int64_t v = v0 + lane();
    bool act = false;
    if (v < g.V) {
      long long ev = g.e[v];
      int32_t hv = g.h[v];
      act = ev > 0 && hv < g.hcap;
      stranded += (ev > 0 && hv == g.hcap) ? 1 : 0;
    }
    wave_append(act, (int32_t)v, a.qout, &a.qcnt[0], a.qcap, a.err);
  }
  stranded = wave_sum_i32(stranded);
  long long bs = group_sum_i64<WB_WAVE>(bscans);
  if (lane() == 0) {
    if (stranded) atomic_add_i64(&a.status[1], stranded);
    if (bs) atomic_add_i64(&a.stats[4], bs);
  }
  grid_barrier(a.bar, nblocks);
  if (gtid == 0) {
    a.status[0] = a.qcnt[0];
    a.status[2] = level;
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

__global__ void k_value(const long long *e, int32_t t, long long *out) { out[0] = e[t] - WB_EXCESS_BIAS; }

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
static unsigned grid1d(int64_t n, int threads = 256, int64_t maxb = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > maxb) b = maxb;
  return (unsigned)b;
}

typedef void (*TileFn)(Graph, SweepQ, int32_t);
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
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(gr_fn(P)), SWEEP_THREADS,
                                                    0) != hipSuccess)
    return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
  return per_cu * prop.multiProcessorCount;
}

// Long rows met in one BFS level produce at most M/chunk + (number of long
// rows) <= M/chunk + V chunk descriptors.
static int64_t chunk_capacity(int32_t V, int64_t Mcap, int chunk) { return Mcap / chunk + V + 16; }

size_t state_bytes(int32_t V, int64_t Mcap, int chunk) {
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  int64_t nchunk = chunk_capacity(V, Mcap, chunk);
  return al(8ull * V) + al(4ull * V) * 6 + al(4ull * nchunk) * 2 + al(4096);
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
  int32_t qcnt[4];
  int32_t fcnt[4];
  int32_t chunk_cnt[2];
  unsigned bar[2];
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
static int run_phase(const SolveConfig &cfg, const Residual &res, State &S, int32_t root, int32_t excl, int P,
                     int gr_blocks, int32_t split_deg, int32_t chunk, hipStream_t st, long long *pinned,
                     PhaseStats *ps, bool second_phase, std::string *err) {
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(S.misc);
  Graph g{res.V, res.V, res.rptr, res.ent, res.rev, S.e, S.h};
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
  ga.split_deg = split_deg;
  ga.chunk = chunk;
  ga.qcap = res.V;
  ga.chunk_cap = (int32_t)std::min<int64_t>(S.nchunk_cap, 0x7fffffff);
  ga.err = misc->err;
  TileFn tfn = tile_fn(P);
  GRFn gfn = gr_fn(P);
  int K = cfg.gr_every_sweeps > 0 ? cfg.gr_every_sweeps : 16;
  const int sweep_blocks = cfg.grid_blocks > 0 ? cfg.grid_blocks : 1024;
  const int block_blocks = 512;
  const int mode = cfg.push_mode == 1 ? 0 : 1;
  auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    hipError_t he = hipMemsetAsync(misc->status, 0, sizeof(misc->status), st);
    if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
    void *args[] = {&ga};
    he = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(gfn), dim3(gr_blocks), dim3(SWEEP_THREADS), args, 0,
                                    st);
    if (he != hipSuccess) { *err = std::string("global relabel launch: ") + hipGetErrorString(he); return 5; }
    ps->global_relabels++;
    he = hipMemcpyAsync(pinned, misc->status, sizeof(misc->status) + sizeof(misc->err), hipMemcpyDeviceToHost, st);
    if (he == hipSuccess) he = hipStreamSynchronize(st);
    if (he != hipSuccess) { *err = std::string("global relabel: ") + hipGetErrorString(he); return 5; }
    const long long active = pinned[0];
    const long long stranded = pinned[1];
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
      SweepQ q;
      q.qin = S.q[j & 1];
      q.qin_cnt = &misc->qcnt[j % 3];
      q.qout = S.q[(j + 1) & 1];
      q.qout_cnt = &misc->qcnt[(j + 1) % 3];
      q.zero_cnt = &misc->qcnt[(j + 2) % 3];
      q.big_v = S.big_v;
      q.big_cnt = &misc->big_cnt[j & 1];
      q.big_cnt_zero = &misc->big_cnt[(j + 1) & 1];
      q.mode = mode;
      q.stats = misc->stats;
      q.qcap = res.V;
      q.err = misc->err;
      if (cfg.time_kernels && S.ev_count < State::kMaxEvents) hipEventRecord(S.ev[S.ev_count][0], st);
      hipLaunchKernelGGL(tfn, dim3(sweep_blocks), dim3(SWEEP_THREADS), 0, st, g, q, split_deg);
      if (cfg.time_kernels && S.ev_count < State::kMaxEvents) {
        hipEventRecord(S.ev[S.ev_count][1], st);
        S.ev_count++;
      }
      hipLaunchKernelGGL(k_sweep_block, dim3(block_blocks), dim3(BLK), 0, st, g, q);
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
  const int P = pick_lanes(cfg, res.V, res.M);
  int32_t split_deg = cfg.split_degree > 0 ? cfg.split_degree : std::max(8 * P, 256);
  const int32_t chunk = 1024;
  int lg = 0;
  while ((1 << lg) < P) lg++;
  int gr_blocks = std::min(gr_blocks_tab[lg], 1024);
  if (gr_blocks < 1) { *err = "cooperative launch not possible"; return 5; }
  rep->lanes = P;
  rep->split_degree = split_deg;
  rep->gr_blocks = gr_blocks;
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(S.misc);
  Graph g{res.V, res.V, res.rptr, res.ent, res.rev, S.e, S.h};
  hipMemsetAsync(S.misc, 0, sizeof(MiscLayout), st);
  hipLaunchKernelGGL(k_init, dim3(grid1d(res.V)), dim3(256), 0, st, g, t);
  hipLaunchKernelGGL(k_preflow, dim3(grid1d(res.M > 0 ? res.M : 1, 256, 4096)), dim3(256), 0, st, g, s);
  auto t0 = std::chrono::steady_clock::now();
  PhaseStats p1{}, p2{};
  int rc = run_phase(cfg, res, S, t, s, P, gr_blocks, split_deg, chunk, st, pinned, &p1, false, err);
  if (rc) return rc;
  hipLaunchKernelGGL(k_value, dim3(1), dim3(1), 0, st, S.e, t, (long long *)dev_value);
  if (dev_side) hipLaunchKernelGGL(k_cut_side, dim3(grid1d(res.V)), dim3(256), 0, st, g, dev_side);
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) { *err = hipGetErrorString(he); return 5; }
  auto t1 = std::chrono::steady_clock::now();
  if (dev_flow) {
    // second phase: return the excess stranded in the source side to s
    hipLaunchKernelGGL(k_add_excess, dim3(1), dim3(1), 0, st, S.e, s, (long long)WB_EXCESS_BIAS);
    rc = run_phase(cfg, res, S, s, t, P, gr_blocks, split_deg, chunk, st, pinned, &p2, true, err);
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
  rep->tile_arc_scans = pinned[0];
  rep->tile_pushes = pinned[1];
  rep->tile_relabels = pinned[2];
  rep->tile_queued = pinned[3];
  rep->arc_scans = pinned[0] + pinned[8];
  rep->pushes = pinned[1] + pinned[9];
  rep->relabels = pinned[2] + pinned[10];
  rep->queued = pinned[3] + pinned[11];
  rep->bfs_scans = pinned[4];
  rep->nonempty_sweeps = pinned[5];
  rep->sweeps = p1.sweeps + p2.sweeps;
  rep->phase2_sweeps = p2.sweeps;
  rep->global_relabels = p1.global_relabels + p2.global_relabels;
  return 0;
}

}  // namespace wb
