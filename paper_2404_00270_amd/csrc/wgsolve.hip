// Persistent batched solve: one workgroup per instance, instances claimed from
// a device work queue (the batched pattern; the paper's Eq. 1 imbalance,
// there across the vertices of one graph, here across instances of uneven
// size: the queue is ordered by decreasing size, so the longest solves start
// first and the workgroups that finish early take the rest).
//
// A workgroup solves its instance whole, in the arena (HBM), with the same
// method as the rounds of launches: an exact backward BFS from the phase's
// target (the global relabel of section 2.2), then sweeps of the active
// vertices (Algorithm 2 with full discharge: a tile of P lanes scans a
// queued vertex's row, pushes along every residual entry to a lower
// neighbour while excess is left, then relabels to one above the lowest
// remaining residual neighbour), until the relabel work since the BFS
// exceeds the instance's budget or no vertex is active; phase 1 ends when no
// vertex with excess reaches t (value and canonical side written), phase 2
// returns stranded excess to s, and the per-arc flows are decoded.  Barriers
// between sweeps and BFS levels are workgroup barriers, not kernel launches
// or grid barriers.  Each instance carries its own schedule: tile width and
// relabel budget (from the autotuner's cache for its shape class, else the
// rule for its mean row length).
//
// One kernel runs for many milliseconds, so the CU's L1 keeps lines across
// sweeps: every read of state that atomics change (residuals, heights,
// excesses) is a device-scope atomic load, served by L2, never a stale L1
// line.  Loops are bounded (rounds 4V + 1024, sweeps per round V + 16, and a
// time limit per instance checked after every sweep); an instance that
// reaches a cap stops in a consistent preflow state and is reported for the
// rounds of launches to finish.
#include "wb_common.h"
#include "wb_kernels.h"

namespace wb {

namespace {

__device__ __forceinline__ int2 ld_ent(const int2 *p) {
  const unsigned long long x = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
  return make_int2((int32_t)(uint32_t)x, (int32_t)(uint32_t)(x >> 32));
}

__device__ __forceinline__ int32_t ld_i32(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ long long ld_i64(const long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_i32(int32_t *p, int32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_i64(long long *p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Residual of entry k (words cr) and of its mate, in either layout.
template <bool RC>
__device__ __forceinline__ int32_t wg_res(const int32_t *rev, int2 cr) {
  return RC && cr.x < 0 ? ld_i32(&rev[cr.y]) : cr.y;
}

template <bool RC>
__device__ __forceinline__ int32_t wg_mate_res(const int2 *ent, const int32_t *rev, int32_t k, int2 cr) {
  if (!RC) return ld_ent(&ent[ld_i32(&rev[k])]).y;
  return cr.x < 0 ? ld_ent(&ent[cr.y]).y : ld_i32(&rev[k]);
}

// Moves d along the entry with push handle hk (see handle_of).
template <bool RC>
__device__ __forceinline__ void wg_move(int2 *ent, int32_t *rev, int32_t hk, int32_t d) {
  if (!RC) {
    atomic_add_i32(&ent[hk].y, -d);
    atomic_add_i32(&ent[rev[hk]].y, d);
  } else if (hk >= 0) {
    atomic_add_i32(&ent[hk].y, -d);
    atomic_add_i32(&rev[hk], d);
  } else {
    atomic_add_i32(&rev[~hk], -d);
    atomic_add_i32(&ent[~hk].y, d);
  }
}

// Appends val to q (capacity cap) at a slot counted in the workgroup's LDS
// counter *cnt, one LDS atomic per wave; an overflow (a bug) raises *bad.
__device__ __forceinline__ void wg_append(bool pred, int32_t val, int32_t *q, int32_t *cnt, int32_t cap, int32_t *bad) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane() == leader) base = atomicAdd(cnt, __popcll(m));
  base = __shfl(base, leader, WB_WAVE);
  if (pred) {
    const int idx = base + __popcll(m & lanemask_lt());
    if (idx < cap) q[idx] = val;
    else *bad = 1;
  }
}

template <int P>
__device__ __forceinline__ long long wg_excl_scan(long long x, long long *total) {
  const int tl = lane() & (P - 1);
  long long incl = x;
#pragma unroll
  for (int dd = 1; dd < P; dd <<= 1) {
    unsigned lo = (unsigned)incl, hi = (unsigned)((unsigned long long)incl >> 32);
    lo = (unsigned)__shfl_up((int)lo, dd, WB_WAVE);
    hi = (unsigned)__shfl_up((int)hi, dd, WB_WAVE);
    const long long y = (long long)(((unsigned long long)hi << 32) | lo);
    if (tl >= dd) incl += y;
  }
  *total = (long long)shfl_u64((unsigned long long)incl, lane() | (P - 1));
  return incl - x;
}

// State of the instance a workgroup is solving.
struct WgSolve {
  int32_t vb, V, s, t;      // arena ids of vertex 0, s and t; V vertices
  int32_t target, other;    // the phase's BFS root and its excluded terminal
  const int2 *rowb;
  int2 *ent;
  int32_t *rev;
  long long *e;
  int32_t *h;
};

struct WgShared {
  int32_t cnt[2];
  int32_t bad;
  int32_t stop;              // the instance ran past its time limit
  int32_t item;
  unsigned long long work;   // relabel work (entries) since the BFS
  long long red[WG_THREADS / WB_WAVE];
};

// One sweep over qin[0, nin): a tile of P lanes per queued vertex, full
// discharge.  Appends to qout (LDS counter sh.cnt[cout]).
template <int P, bool RC>
__device__ void wg_sweep(const WgSolve &c, const int32_t *qin, int32_t nin, int32_t *qout, int cout, WgShared &sh,
                         long long *scans, long long *pushes, long long *relabels) {
  constexpr int UNROLL = 4;
  constexpr int TPW = WB_WAVE / P;
  const int wave = threadIdx.x / WB_WAVE;
  constexpr int NWAVES = WG_THREADS / WB_WAVE;
  const int sub = lane() / P, tl = lane() % P, tbase = lane() & ~(P - 1);
  const bool leader = tl == 0;
  const int32_t hcap = c.V;  // local heights: V is inactive
  for (int32_t b0 = wave * TPW; b0 < nin; b0 += NWAVES * TPW) {  // wave-uniform
    const int32_t i = b0 + sub;
    const bool valid = i < nin;
    int32_t u = 0, beg = 0, end = 0, hu = 0;
    long long e0 = 0;
    if (valid) {
      u = qin[i];
      const int2 rb = c.rowb[u];
      beg = rb.x;
      end = rb.y;
      hu = ld_i32(&c.h[u]);
      if (leader) e0 = ld_i64(&c.e[u]);
    }
    e0 = (long long)shfl_u64((unsigned long long)e0, tbase);
    const bool scan = valid && e0 > 0 && hu < hcap;
    long long erem = scan ? e0 : 0;
    unsigned long long key = WB_KEY_NONE;
    long long nscan = 0;
    for (int32_t kb = beg; scan ? (kb < end && erem > 0) : false; kb += UNROLL * P) {
      int2 cr[UNROLL];
      int32_t rr[UNROLL], hv[UNROLL];
#pragma unroll
      for (int j = 0; j < UNROLL; j++) {
        const int32_t k = kb + j * P + tl;
        cr[j] = k < end ? ld_ent(&c.ent[k]) : make_int2(0, 0);
      }
#pragma unroll
      for (int j = 0; j < UNROLL; j++) rr[j] = wg_res<RC>(c.rev, cr[j]);
#pragma unroll
      for (int j = 0; j < UNROLL; j++) hv[j] = rr[j] > 0 ? ld_i32(&c.h[col_of<RC>(cr[j])]) : 0;
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
            const unsigned long long kk = ((unsigned long long)(unsigned)hv[j] << 32) | (unsigned)(k - beg);
            key = kk < key ? kk : key;
          }
        }
        long long tot;
        const long long before = wg_excl_scan<P>(want, &tot);
        long long take = erem - before;
        take = take < 0 ? 0 : (take > want ? want : take);
        bool app_v = false;
        if (take > 0) {
          wg_move<RC>(c.ent, c.rev, handle_of<RC>(k, cr[j]), (int32_t)take);
          if (v != c.target) {
            const long long oldv = atomic_add_i64(&c.e[v], take);
            app_v = oldv <= 0 && oldv + take > 0 && hv[j] < hcap;
          }
          (*pushes)++;
        }
        wg_append(app_v, v, qout, &sh.cnt[cout], c.V, &sh.bad);
        if (erem > 0 && kb + j * P < end) nscan += P;
        erem -= tot;
      }
    }
    key = group_min<P>(key);
    bool app_u = false;
    if (leader && scan) {
      const int32_t deg = end - beg;
      *scans += nscan < deg ? nscan : deg;
      const long long pushed = e0 - (erem > 0 ? erem : 0);
      long long left = e0;
      if (pushed > 0) left = atomic_add_i64(&c.e[u], -pushed) - pushed;
      if (erem > 0) {
        if (key == WB_KEY_NONE) {
          app_u = true;  // nothing residual visible: next sweep
        } else {
          int32_t nh = (int32_t)(key >> 32) + 1;
          if (nh > hcap) nh = hcap;
          st_i32(&c.h[u], nh);
          (*relabels)++;
          atomicAdd(&sh.work, (unsigned long long)deg);
          app_u = nh < hcap;
        }
      } else {
        app_u = left > 0;
      }
    }
    wg_append(app_u, u, qout, &sh.cnt[cout], c.V, &sh.bad);
  }
}

template <bool RC>
__device__ __forceinline__ void wg_sweep_p(int P, const WgSolve &c, const int32_t *qin, int32_t nin, int32_t *qout,
                                           int cout, WgShared &sh, long long *sc, long long *pu, long long *re) {
  switch (P) {
    case 1: wg_sweep<1, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
    case 4: wg_sweep<4, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
    case 8: wg_sweep<8, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
    case 16: wg_sweep<16, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
    case 32: wg_sweep<32, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
    default: wg_sweep<64, RC>(c, qin, nin, qout, cout, sh, sc, pu, re); break;
  }
}

// One level of the backward BFS: a tile of P lanes per frontier vertex w
// walks w's row and claims every unlabelled v with residual capacity
// toward w (the mate of entry (w, v)).
template <int P, bool RC>
__device__ void wg_bfs_level(const WgSolve &c, const int32_t *fin, int32_t n, int32_t *fout, int nc, int32_t lev,
                             WgShared &sh, long long *bscans) {
  constexpr int TPW = WB_WAVE / P;
  const int wave = threadIdx.x / WB_WAVE, sub = lane() / P, tl = lane() % P;
  for (int32_t b0 = wave * TPW; b0 < n; b0 += (WG_THREADS / WB_WAVE) * TPW) {  // wave-uniform
    const int32_t i = b0 + sub;
    int32_t beg = 0, end = 0;
    if (i < n) {
      const int2 rb = c.rowb[fin[i]];
      beg = rb.x;
      end = rb.y;
      if (tl == 0) *bscans += end - beg;
    }
    for (int32_t kb = beg; kb < end; kb += P) {  // tile-uniform
      const int32_t k = kb + tl;
      bool claimed = false;
      int32_t v = 0;
      if (k < end) {
        const int2 cr = ld_ent(&c.ent[k]);
        v = col_of<RC>(cr);
        if (ld_i32(&c.h[v]) == c.V && wg_mate_res<RC>(c.ent, c.rev, k, cr) > 0)
          claimed = atomicCAS(&c.h[v], c.V, lev) == c.V;
      }
      wg_append(claimed, v, fout, &sh.cnt[nc], c.V, &sh.bad);
    }
  }
}

// Exact heights: backward BFS from c.target over arcs v -> w with residual
// capacity; unreached vertices stay at V (inactive), the excluded terminal
// at V + 1.  Frontiers alternate between fa and fb; tiles of P lanes (the
// instance's tile width, at least 4) expand them.  Returns the levels.
template <bool RC>
__device__ int32_t wg_bfs(const WgSolve &c, int lanes, int32_t *fa, int32_t *fb, WgShared &sh, long long *bscans) {
  const int tid = threadIdx.x;
  for (int32_t x = tid; x < c.V; x += WG_THREADS) {
    const int32_t v = c.vb + x;
    st_i32(&c.h[v], v == c.target ? 0 : (v == c.other ? c.V + 1 : c.V));
  }
  if (tid == 0) {
    fa[0] = c.target;
    sh.cnt[0] = 1;
    sh.cnt[1] = 0;
  }
  __syncthreads();
  int32_t n = sh.cnt[0];
  int32_t lev = 0;
  int cur = 0;
  while (n > 0) {  // at most V levels: every level labels a new vertex
    lev++;
    const int32_t *fin = cur == 0 ? fa : fb;
    int32_t *fout = cur == 0 ? fb : fa;
    const int nc = 1 - cur;
    switch (lanes) {
      case 1:
      case 4: wg_bfs_level<4, RC>(c, fin, n, fout, nc, lev, sh, bscans); break;
      case 8: wg_bfs_level<8, RC>(c, fin, n, fout, nc, lev, sh, bscans); break;
      case 16: wg_bfs_level<16, RC>(c, fin, n, fout, nc, lev, sh, bscans); break;
      default: wg_bfs_level<64, RC>(c, fin, n, fout, nc, lev, sh, bscans); break;
    }
    __syncthreads();
    n = sh.cnt[nc];
    __syncthreads();
    if (tid == 0) sh.cnt[cur] = 0;
    cur = nc;
    __syncthreads();
  }
  return lev;
}

// Sum over the workgroup, returned in every thread (two barriers).
__device__ long long wg_sum(long long x, WgShared &sh) {
  x = group_sum_i64<WB_WAVE>(x);
  __syncthreads();
  if (lane() == 0) sh.red[threadIdx.x / WB_WAVE] = x;
  __syncthreads();
  long long t = 0;
#pragma unroll
  for (int w = 0; w < WG_THREADS / WB_WAVE; w++) t += sh.red[w];
  return t;
}

template <bool RC>
__device__ int32_t wg_solve_one(const WgArgs &a, const WgInst &d, WgShared &sh, long long *st) {
  const int tid = threadIdx.x;
  WgSolve c;
  c.vb = d.vbase;
  c.V = d.V;
  c.s = d.s;
  c.t = d.t;
  c.rowb = a.rowb;
  c.ent = a.ent;
  c.rev = a.rev;
  c.e = a.e;
  c.h = a.h;
  int32_t *qa = a.qa + d.vbase, *qb = a.qb + d.vbase;  // this instance's slices: V entries each
  const int64_t M = (int64_t)a.rowb[d.vbase + d.V - 1].y - a.rowb[d.vbase].x;
  const unsigned long long budget =
      (unsigned long long)((double)(d.budget_pm > 0 ? d.budget_pm : 1000) / 1000.0 * (double)(d.V + M)) + 1;
  const int32_t round_cap = a.round_cap > 0 ? a.round_cap : 4 * d.V + 1024, sweep_cap = d.V + 16;
  const int P = d.lanes;
  const long long t_start = tid == 0 ? (long long)wall_clock64() : 0;  // read by thread 0 only
  int phase = 1, rounds = 0;
  for (;;) {  // every branch is uniform over the workgroup
    c.target = phase == 1 ? d.t : d.s;
    c.other = phase == 1 ? d.s : d.t;
    if (tid == 0) sh.bad = 0;
    wg_bfs<RC>(c, d.lanes, qa, qb, sh, &st[5]);
    if (tid == 0) st[4]++;
    // active vertices: excess and a path to the target
    if (tid == 0) sh.cnt[0] = 0;
    __syncthreads();
    for (int32_t x0 = tid - lane(); x0 < d.V; x0 += WG_THREADS) {  // wave-uniform
      const int32_t x = x0 + lane();
      bool act = false;
      if (x < d.V) {
        const int32_t v = d.vbase + x;
        act = v != d.s && v != d.t && ld_i64(&c.e[v]) > 0 && ld_i32(&c.h[v]) < d.V;
      }
      wg_append(act, d.vbase + x, qa, &sh.cnt[0], d.V, &sh.bad);
    }
    __syncthreads();
    int32_t na = sh.cnt[0];
    if (sh.bad) return phase == 1 ? 2 : 3;  // a list overflowed (cannot happen): leave it to the rounds
    if (na == 0) {
      if (phase == 1) {
        // maximum preflow: value = flow into t, side = vertices that reach t
        const int2 rt = a.rowb[d.t];
        long long acc = 0;
        for (int32_t k = rt.x + tid; k < rt.y; k += WG_THREADS)
          acc += (long long)wg_res<RC>(a.rev, ld_ent(&a.ent[k])) - (long long)a.cap0[k];
        acc = wg_sum(acc, sh);
        if (tid == 0 && d.value) *d.value = acc;
        if (d.side)
          for (int32_t x = tid; x < d.V; x += WG_THREADS) d.side[x] = ld_i32(&c.h[d.vbase + x]) < d.V ? 1 : 0;
        if (!d.flow) break;
        if (tid == 0) atomic_add_i64(&c.e[d.s], WB_EXCESS_BIAS);  // s never tests active in phase 2
        __syncthreads();
        phase = 2;
        continue;
      }
      break;
    }
    if (++rounds > round_cap) return phase == 1 ? 2 : 3;
    if (tid == 0) sh.work = 0;
    int cin = 0;
    for (int32_t sw = 0; sw < sweep_cap && na > 0; sw++) {
      int32_t *qin = cin == 0 ? qa : qb, *qout = cin == 0 ? qb : qa;
      if (tid == 0) sh.cnt[1 - cin] = 0;
      __syncthreads();
      wg_sweep_p<RC>(P, c, qin, na, qout, 1 - cin, sh, &st[0], &st[1], &st[2]);
      if (tid == 0) {
        st[3]++;
        sh.stop = a.max_ticks > 0 && (long long)wall_clock64() - t_start > a.max_ticks;
      }
      __syncthreads();
      na = sh.cnt[1 - cin];
      const bool over = sh.work > budget, stop = sh.stop != 0;
      __syncthreads();
      cin = 1 - cin;
      // a list overflow (cannot happen) or the time limit: the state after a
      // whole sweep is a valid preflow, which the rounds finish
      if (sh.bad || stop) return phase == 1 ? 2 : 3;
      if (over) break;
    }
  }
  // per-arc flows from the final residuals
  if (d.flow) {
    if (RC) {
      for (int64_t i = tid; i < d.E; i += WG_THREADS) d.flow[i] = ld_i32(&a.rev[a.arc2ent[d.abase + i]]);
    } else {
      for (int64_t i = tid; i < d.E; i += WG_THREADS) {
        const int32_t j = a.arc2ent[d.abase + i];
        int32_t f = 0;
        if (j >= 0) {
          const long long x = (long long)a.cap0[j] - (long long)ld_ent(&a.ent[j]).y - (long long)a.pbefore[d.abase + i];
          const long long cc = a.acap[d.abase + i];
          f = (int32_t)(x < 0 ? 0 : (x > cc ? cc : x));
        }
        d.flow[i] = f;
      }
    }
  }
  // finished: inactive, no excess (t keeps its bias), as a solved instance
  for (int32_t x = tid; x < d.V; x += WG_THREADS) {
    const int32_t v = d.vbase + x;
    st_i64(&c.e[v], v == d.t ? WB_EXCESS_BIAS : 0);
    st_i32(&c.h[v], HCAP);
  }
  return 1;
}

// Next list entry for this workgroup, or -1.  Batch mode (no tail): a plain
// claim.  Persistent mode: entries are published while the kernel runs;
// the workgroup waits (sleeping) for one until `close` is set or idle_ticks
// of the 100 MHz clock pass without one, so every workgroup exits.
__device__ int32_t wg_claim(const WgArgs &a) {
  if (!a.tail) {
    const int32_t i = atomicAdd(a.head, 1);
    return i < a.n ? i : -1;
  }
  const long long t0 = (long long)wall_clock64();
  for (;;) {
    const int32_t tail = __hip_atomic_load(a.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    int32_t head = ld_i32(a.head);
    while (head < tail) {
      if (__hip_atomic_compare_exchange_strong(a.head, &head, head + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT))
        return head;
    }
    if (a.close && ld_i32(a.close) != 0) return -1;
    if ((long long)wall_clock64() - t0 > a.idle_ticks) return -1;
    __builtin_amdgcn_s_sleep(8);
  }
}

}  // namespace

template <bool RC>
__global__ void __launch_bounds__(WG_THREADS) k_wg_solve(WgArgs a) {
  __shared__ WgShared sh;
  long long st[6] = {0, 0, 0, 0, 0, 0};  // scans, pushes, relabels, sweeps, BFS rounds, BFS scans
  for (;;) {
    if (threadIdx.x == 0) sh.item = wg_claim(a);
    __syncthreads();
    const int32_t item = sh.item;
    __syncthreads();
    if (item < 0) break;
    const int32_t slot = a.ring > 0 ? item % a.ring : item;
    const WgInst d = a.L[slot];
    const int32_t r = wg_solve_one<RC>(a, d, sh, st);
    __syncthreads();
    // publishes the instance's outputs (written by every thread before the
    // barrier) together with its result
    if (threadIdx.x == 0) __hip_atomic_store(&a.result[slot], r, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  // counters: one atomic per workgroup and counter
  for (int k = 0; k < 6; k++) {
    const long long x = wg_sum(st[k], sh);
    if (threadIdx.x == 0 && x && a.stats) atomic_add_i64(&a.stats[k], x);
  }
}

__global__ void __launch_bounds__(256) k_pk_publish(const WgInst *staged, int32_t n, WgInst *ring, int32_t R,
                                                    int32_t *result, int32_t *tail) {
  const int32_t t0 = ld_i32(tail);
  for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const int32_t slot = (int32_t)(((int64_t)t0 + i) % R);
    ring[slot] = staged[i];
    st_i32(&result[slot], 0);
  }
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(tail, t0 + n, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

void launch_pk_publish(hipStream_t st, const WgInst *staged, int32_t n, WgInst *ring, int32_t R, int32_t *result,
                       int32_t *tail) {
  hipLaunchKernelGGL(k_pk_publish, dim3(1), dim3(256), 0, st, staged, n, ring, R, result, tail);
}

void launch_wg_solve(bool rc, int blocks, hipStream_t st, const WgArgs &a) {
  if (rc) hipLaunchKernelGGL(k_wg_solve<true>, dim3(blocks), dim3(WG_THREADS), 0, st, a);
  else hipLaunchKernelGGL(k_wg_solve<false>, dim3(blocks), dim3(WG_THREADS), 0, st, a);
}

}  // namespace wb
