// Host engine (wb_engine.h) and its per-instance kernels.
//
// Every resident instance owns a contiguous vertex range, entry range and arc
// range of the arena.  Kernels address vertices and entries by arena id, so
// the residual graphs of all resident instances form one disjoint union: a
// sweep or a global relabel serves every instance at once.  Heights carry a
// per-instance base HCAP - V_i, so "h >= HCAP" means "local height >= V_i"
// (inactive) for every instance alike (Algorithm 1's deactivation at |V|).
//
// Per instance the phases are: 1, maximum preflow (sink t is the BFS root,
// source s excluded) until no active vertex is left; then the flow value and
// the cut side are written; 2, if per-arc flows are wanted, the stranded
// excess returns to s (s is the root, t excluded); then the flows are
// decoded; 3, done and released.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../include/wbpr.h"
#include "wb_common.h"
#include "wb_engine.h"

namespace wb {

// ------------------------------------------------------------ range alloc
void RangeAlloc::reset(int64_t cap) {
  free_.clear();
  cap_ = cap;
  free_total_ = cap;
  if (cap > 0) free_[0] = cap;
}

int64_t RangeAlloc::alloc(int64_t n) {
  if (n <= 0) return 0;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= n) {
      const int64_t at = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[at + n] = len - n;
      free_total_ -= n;
      return at;
    }
  }
  return -1;
}

void RangeAlloc::release(int64_t at, int64_t n) {
  if (n <= 0) return;
  free_total_ += n;
  auto it = free_.emplace(at, n).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

void RangeAlloc::shrink(int64_t at, int64_t n_old, int64_t n_new) {
  if (n_new < n_old) release(at + n_new, n_old - n_new);
}

int64_t RangeAlloc::largest_free() const {
  int64_t b = 0;
  for (const auto &kv : free_) b = std::max(b, kv.second);
  return b;
}

// ------------------------------------------------------ per-instance kernels
struct InstDev {
  int32_t vbase, V, s, t;  // s, t: arena ids
  int64_t abase, E;
  long long *value;
  int32_t *flow;
  uint8_t *side;
  int64_t pad;  // every list slice also holds WgInst entries of the same size
};

enum InstKernel {
  IK_INIT = 0, IK_PREFLOW, IK_VALUE_ZERO, IK_VALUE, IK_SIDE, IK_PHASE2, IK_DECODE, IK_RELEASE, IK_PARK, IK_MAXDEG,
  IK_SMALL,  // list slice of the LDS-resident solve (k_small_solve, not k_inst)
  IK_WG,     // list slice of the persistent workgroup-per-instance solve (k_wg_solve)
  IK_COUNT
};

struct InstArgs {
  const InstDev *L;
  int2 *rowb;
  int2 *ent;
  int32_t *rev;         // BCSR: mates; RCSR: flows (at forward entries)
  const int32_t *cap0;
  const int32_t *arc2ent;
  const int32_t *pbefore;
  const int32_t *acap;
  long long *e;
  int32_t *h;
  int32_t *inst_of;
  const int32_t *slot;  // [n] instance slot of list entry i (IK_INIT)
  int32_t *maxdeg;      // [n] longest row of list entry i, terminals excluded (IK_MAXDEG)
  int32_t rcsr;         // rows in the RCSR layout
};

// Residual of entry k whose words are cr, in either layout (one-off
// per-instance kernels: a runtime branch).
__device__ __forceinline__ int32_t inst_res(const InstArgs &a, int2 cr) {
  return a.rcsr && cr.x < 0 ? a.rev[cr.y] : cr.y;
}

// Whole solve of one small instance by one workgroup, its residual graph in
// LDS (the batched pattern for instances of up to about a thousand
// vertices): starts from the preflow state in the arena, alternates a BFS
// from the phase's target (exact heights, as the global relabel) with sweeps
// of single pushes or relabels (Algorithms 1-2, one thread per active
// vertex, LDS atomics), writes the value and the sink side when phase 1
// ends, returns stranded excess to s when flows are wanted (phase 2), and
// writes the final residuals back for the flow decode.  result[i]: 1 solved,
// 0 not taken (does not fit the LDS budget), 2 gave up at the round cap.
// Only a solved instance writes anything back to the arena (value and side
// are rewritten by whoever finishes it), so the other two leave it in its
// preflow state for the rounds of launches.
constexpr int SMALL_THREADS = 1024;

struct SmallArgs {
  const InstDev *L;
  const int2 *rowb;
  int2 *ent;
  const int32_t *rev;
  const int32_t *cap0;
  long long *e;
  int32_t *h;
  int32_t *result;
  long long *stats;  // [0] arc scans of the sweeps, [2] relabels, [1] pushes (as the tile kernel's)
  int32_t lds_bytes;
  int32_t round_cap;  // BFS rounds before giving up (0: 4V + 1024)
};

__device__ __forceinline__ size_t small_al(size_t x) { return (x + 15) & ~(size_t)15; }

__global__ void __launch_bounds__(SMALL_THREADS) k_small_solve(SmallArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  __shared__ int32_t s_cnt[2];
  __shared__ long long s_part[SMALL_THREADS / WB_WAVE];
  const InstDev d = a.L[blockIdx.x];
  const int tid = threadIdx.x;
  const int32_t V = d.V;
  const int64_t mb = a.rowb[d.vbase].x;
  const int64_t M = (int64_t)a.rowb[d.vbase + V - 1].y - mb;
  // LDS: row starts, excess, heights, two vertex lists, residuals, columns, mates
  const size_t need = small_al(4 * ((size_t)V + 1)) + small_al(8 * (size_t)V) + small_al(4 * (size_t)V) +
                      2 * small_al(2 * (size_t)V) + small_al(4 * (size_t)M) + 2 * small_al(2 * (size_t)M);
  if (V > 65535 || M > 65535 || need > (size_t)a.lds_bytes) {  // uniform over the workgroup
    if (tid == 0) a.result[blockIdx.x] = 0;
    return;
  }
  unsigned char *p = lds;
  int32_t *rp = (int32_t *)p;           p += small_al(4 * ((size_t)V + 1));
  long long *ex = (long long *)p;       p += small_al(8 * (size_t)V);
  int32_t *ht = (int32_t *)p;           p += small_al(4 * (size_t)V);
  uint16_t *qa = (uint16_t *)p;         p += small_al(2 * (size_t)V);
  uint16_t *qb = (uint16_t *)p;         p += small_al(2 * (size_t)V);
  int32_t *res = (int32_t *)p;          p += small_al(4 * (size_t)M);
  uint16_t *col = (uint16_t *)p;        p += small_al(2 * (size_t)M);
  uint16_t *rv = (uint16_t *)p;
  const int32_t ss = d.s - d.vbase, tt = d.t - d.vbase;
  for (int32_t x = tid; x < V; x += SMALL_THREADS) {
    rp[x] = (int32_t)(a.rowb[d.vbase + x].x - mb);
    ex[x] = (x == ss || x == tt) ? 0 : a.e[d.vbase + x];
  }
  if (tid == 0) rp[V] = (int32_t)M;
  for (int64_t k = tid; k < M; k += SMALL_THREADS) {
    const int2 c = a.ent[mb + k];
    col[k] = (uint16_t)(c.x - d.vbase);
    res[k] = c.y;
    rv[k] = (uint16_t)(a.rev[mb + k] - mb);
  }
  __syncthreads();
  const bool two_phases = d.flow != nullptr;
  long long scans = 0, pushes = 0, relabels = 0;
  const int32_t round_cap = a.round_cap > 0 ? a.round_cap : 4 * V + 1024, sweep_cap = V + 16;
  int phase = 1, rounds = 0;
  bool ok = true;
  for (;;) {  // every branch below is uniform over the workgroup
    const int32_t target = phase == 1 ? tt : ss, other = phase == 1 ? ss : tt;
    // exact heights: BFS from the target over arcs v -> w with residual > 0
    for (int32_t x = tid; x < V; x += SMALL_THREADS) ht[x] = x == target ? 0 : (x == other ? V + 1 : V);
    if (tid == 0) {
      qa[0] = (uint16_t)target;
      s_cnt[0] = 1;
    }
    __syncthreads();
    uint16_t *fa = qa, *fb = qb;
    int32_t nq = s_cnt[0];
    for (int32_t lev = 1; nq > 0; lev++) {
      __syncthreads();
      if (tid == 0) s_cnt[0] = 0;
      __syncthreads();
      for (int32_t i = tid; i < nq; i += SMALL_THREADS) {
        const int32_t w = fa[i];
        for (int32_t k = rp[w]; k < rp[w + 1]; k++) {
          const int32_t v = col[k];
          if (ht[v] == V && res[rv[k]] > 0 && atomicCAS(&ht[v], V, lev) == V) fb[atomicAdd(&s_cnt[0], 1)] = (uint16_t)v;
        }
      }
      __syncthreads();
      nq = s_cnt[0];
      uint16_t *tq = fa;
      fa = fb;
      fb = tq;
    }
    __syncthreads();
    // active vertices: excess and a path to the target
    if (tid == 0) s_cnt[1] = 0;
    __syncthreads();
    for (int32_t x = tid; x < V; x += SMALL_THREADS)
      if (x != ss && x != tt && ex[x] > 0 && ht[x] < V) qa[atomicAdd(&s_cnt[1], 1)] = (uint16_t)x;
    __syncthreads();
    int32_t na = s_cnt[1];
    if (na == 0) {
      if (phase == 1) {
        // maximum preflow: sink side = vertices that still reach t; value =
        // flow into t = sum over t's row of (residual - initial capacity)
        if (d.side)
          for (int32_t x = tid; x < V; x += SMALL_THREADS) d.side[x] = ht[x] < V ? 1 : 0;
        long long acc = 0;
        for (int32_t k = rp[tt] + tid; k < rp[tt + 1]; k += SMALL_THREADS)
          acc += (long long)res[k] - (long long)a.cap0[mb + k];
        acc = group_sum_i64<WB_WAVE>(acc);
        if (lane() == 0) s_part[tid / WB_WAVE] = acc;
        __syncthreads();
        if (tid == 0 && d.value) {
          long long tot = 0;
          for (int w = 0; w < SMALL_THREADS / WB_WAVE; w++) tot += s_part[w];
          *d.value = tot;
        }
        if (!two_phases) break;
        phase = 2;  // return stranded excess to s
        continue;
      }
      break;
    }
    if (++rounds > round_cap) {
      ok = false;
      break;
    }
    // sweeps: one push to the lowest residual neighbour, else a relabel
    for (int32_t sw = 0; sw < sweep_cap && na > 0; sw++) {
      for (int32_t i = tid; i < na; i += SMALL_THREADS) {
        const int32_t u = qa[i];
        const long long eu = ex[u];
        const int32_t hu = ht[u];
        if (eu <= 0 || hu >= V) continue;
        int32_t hmin = 0x7fffffff, kmin = -1;
        scans += rp[u + 1] - rp[u];
        for (int32_t k = rp[u]; k < rp[u + 1]; k++)
          if (res[k] > 0) {
            const int32_t hv = ht[col[k]];
            if (hv < hmin) {
              hmin = hv;
              kmin = k;
            }
          }
        if (kmin < 0) continue;
        if (hu > hmin) {
          const int32_t r = res[kmin];
          const int32_t dd = (int32_t)(eu < (long long)r ? eu : (long long)r);
          atomicSub(&res[kmin], dd);
          atomicAdd(&res[rv[kmin]], dd);
          atomicAdd((unsigned long long *)&ex[u], (unsigned long long)(-(long long)dd));
          atomicAdd((unsigned long long *)&ex[col[kmin]], (unsigned long long)(long long)dd);
          pushes++;
        } else {
          ht[u] = hmin + 1 < V ? hmin + 1 : V;
          relabels++;
        }
      }
      __syncthreads();
      if (tid == 0) s_cnt[1] = 0;
      __syncthreads();
      for (int32_t x = tid; x < V; x += SMALL_THREADS)
        if (x != ss && x != tt && ex[x] > 0 && ht[x] < V) qa[atomicAdd(&s_cnt[1], 1)] = (uint16_t)x;
      __syncthreads();
      na = s_cnt[1];
      __syncthreads();
    }
  }
  __syncthreads();
  if (ok) {
    for (int64_t k = tid; k < M; k += SMALL_THREADS) a.ent[mb + k].y = res[k];
    for (int32_t x = tid; x < V; x += SMALL_THREADS) {
      a.e[d.vbase + x] = x == tt ? WB_EXCESS_BIAS : 0;
      a.h[d.vbase + x] = HCAP;
    }
  }
  scans = group_sum_i64<WB_WAVE>(scans);
  pushes = group_sum_i64<WB_WAVE>(pushes);
  relabels = group_sum_i64<WB_WAVE>(relabels);
  if (lane() == 0) {
    if (scans) atomic_add_i64(&a.stats[0], scans);
    if (pushes) atomic_add_i64(&a.stats[1], pushes);
    if (relabels) atomic_add_i64(&a.stats[2], relabels);
  }
  if (tid == 0) a.result[blockIdx.x] = ok ? 1 : 2;
}

// blockIdx.y selects the instance of the list; blockIdx.x strides its range.
__global__ void k_inst(InstArgs a, int which) {
  const InstDev d = a.L[blockIdx.y];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  switch (which) {
    case IK_INIT:
      for (int64_t x = tid; x < d.V; x += nth) {
        const int32_t v = d.vbase + (int32_t)x;
        a.e[v] = v == d.t ? WB_EXCESS_BIAS : 0;
        a.h[v] = 0;
        a.inst_of[v] = a.slot[blockIdx.y];
      }
      break;
    case IK_PREFLOW: {  // Algorithm 1, step 0: saturate every residual entry of s
      const int2 rb = a.rowb[d.s];
      for (int64_t k = rb.x + tid; k < rb.y; k += nth) {
        const int2 cr = a.ent[k];
        if (!a.rcsr) {
          if (cr.y > 0) {
            a.ent[k].y = 0;
            atomic_add_i32(&a.ent[a.rev[k]].y, cr.y);
            atomic_add_i64(&a.e[cr.x], (long long)cr.y);
          }
        } else if (cr.x >= 0 && cr.y > 0) {
          // RCSR: only forward entries of s have residual at the start (the
          // flow on s's in-arcs, their reverse entries' residual, is 0)
          a.ent[k].y = 0;
          a.rev[k] = cr.y;
          atomic_add_i64(&a.e[cr.x], (long long)cr.y);
        }
      }
      break;
    }
    case IK_VALUE_ZERO:
      if (tid == 0 && d.value) *d.value = 0;
      break;
    case IK_VALUE: {
      // value = total flow into t = sum over t's row of (c_f(t,w) - c(t,w)):
      // every push w -> t raised the mate residual c_f(t,w) by the amount
      // pushed, and nothing is ever pushed out of t
      __shared__ long long s_part[256 / WB_WAVE];
      const int2 rb = a.rowb[d.t];
      long long acc = 0;
      for (int64_t k = rb.x + tid; k < rb.y; k += nth) acc += (long long)inst_res(a, a.ent[k]) - (long long)a.cap0[k];
      acc = group_sum_i64<WB_WAVE>(acc);
      if (lane() == 0) s_part[threadIdx.x / WB_WAVE] = acc;
      __syncthreads();
      if (threadIdx.x == 0 && d.value) {
        long long tot = 0;
        for (int i = 0; i < (int)(blockDim.x / WB_WAVE); i++) tot += s_part[i];
        if (tot) atomic_add_i64(d.value, tot);
      }
      break;
    }
    case IK_SIDE:  // sink side: v still reaches t (labelled by the last relabel)
      if (d.side)
        for (int64_t x = tid; x < d.V; x += nth) d.side[x] = a.h[d.vbase + x] < HCAP ? 1 : 0;
      break;
    case IK_PHASE2:
      if (tid == 0) a.e[d.s] += WB_EXCESS_BIAS;
      break;
    case IK_DECODE:
      // per-arc flow from the merged net flow of the ordered pair (u,v):
      // parallel arcs u->v are filled in input order up to their capacities
      if (d.flow && a.rcsr) {  // RCSR: every arc has its own flow word
        for (int64_t i = tid; i < d.E; i += nth) d.flow[i] = a.rev[a.arc2ent[d.abase + i]];
      } else if (d.flow)
        for (int64_t i = tid; i < d.E; i += nth) {
          const int32_t j = a.arc2ent[d.abase + i];
          int32_t f = 0;
          if (j >= 0) {
            long long x = (long long)a.cap0[j] - (long long)a.ent[j].y - (long long)a.pbefore[d.abase + i];
            const long long c = a.acap[d.abase + i];
            f = (int32_t)(x < 0 ? 0 : (x > c ? c : x));
          }
          d.flow[i] = f;
        }
      break;
    case IK_MAXDEG: {  // longest row a sweep can meet: terminals are never queued
      __shared__ int s_m;
      if (threadIdx.x == 0) s_m = 0;
      __syncthreads();
      int32_t m = 0;
      for (int64_t x = tid; x < d.V; x += nth) {
        const int32_t v = d.vbase + (int32_t)x;
        if (v == d.s || v == d.t) continue;
        const int2 rb = a.rowb[v];
        m = max(m, rb.y - rb.x);
      }
#pragma unroll
      for (int o = WB_WAVE / 2; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, WB_WAVE));
      // one device atomic per workgroup (same-address atomics serialise)
      if (lane() == 0 && m > 0) atomicMax(&s_m, m);
      __syncthreads();
      if (threadIdx.x == 0 && s_m > 0) atomicMax(&a.maxdeg[blockIdx.y], s_m);
      break;
    }
    case IK_RELEASE:
    case IK_PARK:  // a kept graph between solves: rows stay, nothing active
      for (int64_t x = tid; x < d.V; x += nth) {
        const int32_t v = d.vbase + (int32_t)x;
        a.e[v] = 0;
        a.h[v] = HCAP;
        a.inst_of[v] = -1;
        if (which == IK_RELEASE) a.rowb[v] = make_int2(0, 0);
      }
      break;
  }
}

// Packs n local CSRs into one union CSR: vertex ids offset by voff[i], arcs
// by eoff[i]; checks each instance's row pointers and columns (bad[i]).
__global__ void k_union_rows(int32_t n, const int32_t *voff, const int64_t *eoff, const int64_t *rp_packed,
                             int64_t *rp_union, int32_t *bad) {
  const int32_t Vt = voff[n];
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= Vt; x += (int64_t)gridDim.x * blockDim.x) {
    if (x == Vt) {
      rp_union[x] = eoff[n];
      continue;
    }
    int32_t lo = 0, hi = n - 1;  // last instance with voff <= x
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (voff[mid] <= x) lo = mid; else hi = mid - 1;
    }
    const int32_t i = lo;
    const int64_t local = x - voff[i];
    const int64_t base = (int64_t)voff[i] + i;  // instance i's row pointers start here
    const int64_t r0 = rp_packed[base + local], r1 = rp_packed[base + local + 1];
    const int64_t Ei = eoff[i + 1] - eoff[i];
    bool ok = r0 <= r1 && r0 >= 0 && r1 <= Ei;
    if (local == 0 && r0 != 0) ok = false;
    if (x + 1 == voff[i + 1] && r1 != Ei) ok = false;
    if (!ok) atomic_add_i32(&bad[i], 1);
    rp_union[x] = eoff[i] + (r0 < 0 ? 0 : (r0 > Ei ? Ei : r0));
  }
}

__global__ void k_union_cols(int32_t n, const int32_t *voff, const int64_t *eoff, const int32_t *col_packed,
                             int32_t *col_union, int32_t *bad) {
  const int64_t Et = eoff[n];
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < Et; k += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = n - 1;  // last instance with eoff <= k
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (eoff[mid] <= k) lo = mid; else hi = mid - 1;
    }
    const int32_t i = lo;
    const int32_t c = col_packed[k];
    const int32_t Vi = voff[i + 1] - voff[i];
    if (c < 0 || c >= Vi) {
      atomic_add_i32(&bad[i], 1);
      col_union[k] = voff[i];  // any in-range id; the group is rejected
    } else {
      col_union[k] = voff[i] + c;
    }
  }
}

// ---------------------------------------------------------------- layout
namespace {
struct MiscLayout {
  long long stats[16];
  long long status[4];
  int32_t err[2];
  int32_t qcnt[4];
  int32_t fcnt[4];
  int32_t chunk_cnt[2];
  int32_t big_cnt[2];
  int32_t mid_cnt[2];
  int32_t task_cnt[2];
  int32_t bucnt[4];
  int32_t halt[2];
  long long rwork;
  long long rwork_at_gr;
  unsigned bar[WB_BAR_WORDS];
  long long fedges[4];
  int32_t sink;
  int32_t log_n;
  long long budget;
  int32_t scan_cnt;  // full-scan queue count
  int32_t span;      // end of the highest resident vertex range
  int32_t stag[2];   // stagnation state of the sweeps
  int32_t wtrace_n;  // per-wave trace records written this solve
  int32_t sweep_no;  // sweeps that ran this solve (trace only)
  int32_t gap[4];    // gap heuristic state (lowest empty height, root height, heights counted)
  int32_t wg_head[2];  // claim counter of the persistent per-instance kernel
  int32_t pk_head;     // persistent mode (live admission): entries claimed ...
  int32_t pk_tail;     // ... and published
  long long wg_stats[6];  // its scans, pushes, relabels, sweeps, BFS rounds, BFS scans
  unsigned long long dbg[2];  // debug_checks: entries, vertices violating the preflow invariants
  alignas(128) long long part[PART_SLOTS * PART_WORDS];  // sweep kernels' per-workgroup counters
};

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

int64_t chunk_capacity(int64_t Vcap, int64_t Mcap, int chunk) { return Mcap / chunk + Vcap + 16; }

// The medium-row list doubles as the relabel's four bitmaps.
int64_t mid_words(int64_t Vcap) { return std::max<int64_t>(Vcap, 4 * ((Vcap + 31) / 32)); }

// Long-row chunk tasks of one sweep: every deferred vertex has
// ceil(deg / CHUNK) <= deg / CHUNK + 1 tasks.
int64_t task_capacity(int64_t Vcap, int64_t Mcap) { return Vcap + Mcap / CHUNK + 64; }

unsigned grid1d(int64_t n, int threads = 256, int64_t maxb = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > maxb) b = maxb;
  return (unsigned)b;
}

double gr_beta_env() {
  static double beta = -1;
  if (beta < 0) {
    const char *e = std::getenv("WBPR_GR_BETA");
    beta = e ? std::atof(e) : 1.0;
    if (!(beta > 0)) beta = 1.0;
  }
  return beta;
}

int log_level() {
  static int lvl = -1;
  if (lvl < 0) {
    const char *e = std::getenv("WBPR_LOG");
    lvl = e ? std::atoi(e) : 0;
  }
  return lvl;
}

constexpr int kListKinds = IK_COUNT;  // separate staging per per-instance kernel kind
constexpr int kSweepLogCap = 16384;  // sweep-log records kept (WBPR_LOG >= 2)
constexpr size_t kPinnedHeader = 4096;
}  // namespace

size_t Engine::arena_bytes(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap) {
  const int64_t nch = chunk_capacity(Vcap, Mcap, BFS_CHUNK);
  size_t b = 0;
  b += al(8 * (size_t)Vcap);                 // rowb
  b += al(8 * (size_t)Mcap);                 // ent
  b += 2 * al(4 * (size_t)Mcap);             // rev, cap0
  b += 3 * al(4 * (size_t)Ecap);             // arc2ent, pbefore, acap
  b += al(8 * (size_t)Vcap);                 // e
  b += 4 * al(4 * (size_t)Vcap);             // h, inst_of, q0, q1
  b += al(4 * (size_t)mid_words(Vcap));      // medium-row list (relabel: bitmaps)
  b += 2 * al(4 * (size_t)Vcap);             // BFS frontiers fq0, fq1
  b += 2 * al(4 * (size_t)Vcap);             // long-row list, lr_cnt
  b += 2 * al(4 * (size_t)task_capacity(Vcap, Mcap));  // chunk tasks
  b += al((size_t)Vcap);                     // vis
  b += al(4 * (size_t)GAP_BINS);             // gap heuristic: vertices per height
  b += al(8 * (size_t)nch);                  // BFS chunk descriptors (sweeps: lr_key)
  b += 5 * al(4 * (size_t)ncap) + al(8 * (size_t)ncap);  // active, stranded, roots, root_h, excl; debug terminals
  b += al(sizeof(InstDev) * (size_t)ncap * kListKinds + 4 * (size_t)ncap);  // lists + slots
  b += 2 * al(sizeof(WgInst) * (size_t)ncap) + al(4 * (size_t)ncap);  // persistent ring, staging, results
  b += al(sizeof(MiscLayout));
  b += al(6 * 4 * (size_t)kSweepLogCap);     // sweep log (diagnostics)
  return b;
}

size_t Engine::scratch_bytes(int64_t V, int64_t E, int32_t n) {
  size_t b = build_scratch_bytes((int32_t)V, E);
  b += al(8 * ((size_t)V + 1)) + al(4 * (size_t)(E > 0 ? E : 1));  // union CSR
  b += al(4 * ((size_t)n + 1)) + al(8 * ((size_t)n + 1)) + al(4 * (size_t)n);  // voff, eoff, bad
  b += al(sizeof(BuildStatus));
  return b;
}

Engine::Engine(int device) : device_(device) {
  for (int lg = 2; lg <= 6; lg++) gr_blocks_[lg] = gr_max_blocks(device, 1 << lg);
}

Engine::~Engine() {
  drop_graphs();
  for (auto &e : ev_) hipEventDestroy(e);
  for (auto &e : fork_ev_) hipEventDestroy(e);
  if (side_) hipStreamDestroy(side_);
  if (wtrace_) hipFree(wtrace_);
  if (pk_ev_) {
    if (pk_launched_) hipEventSynchronize(pk_ev_);
    hipEventDestroy(pk_ev_);
  }
  if (!external_) {
    if (arena_) hipFree(arena_);
    if (scratch_) hipFree(scratch_);
    if (pin_) hipHostFree(pin_);
  }
}

void Engine::set_external(void *base, size_t bytes) {
  external_ = true;
  ext_base_ = base;
  ext_bytes_ = bytes;
  arena_ = scratch_ = nullptr;
  arena_n_ = scratch_n_ = 0;
  Vcap_ = Mcap_ = Ecap_ = 0;
  ncap_ = 0;
  sV_ = sE_ = 0;
  sn_ = 0;
}

void Engine::set_config(const SolveConfig &cfg) {
  cfg_ = cfg;
  drop_graphs();
  next_K_ = 12;
}

void Engine::drop_graphs() {
  for (auto &kv : graphs_) {
    hipGraphExecDestroy(kv.second.second);
    hipGraphDestroy(kv.second.first);
  }
  graphs_.clear();
}

int Engine::reserve(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap, int64_t sV, int64_t sE, int32_t sn,
                    std::string *err) {
  Vcap = std::max<int64_t>(Vcap, 2);
  Mcap = std::max<int64_t>(Mcap, 2);
  Ecap = std::max<int64_t>(Ecap, 1);
  ncap = std::max<int32_t>(ncap, 1);
  if (Vcap >= (1ll << 30) || Mcap >= (1ll << 31) - 1 || Ecap >= (1ll << 31) - 1) {
    *err = "arena capacity beyond the 32-bit index limits";
    return WBPR_ETOOBIG;
  }
  if (external_) {
    if (resident_ > 0) {
      *err = "arena cannot change while instances are resident";
      return WBPR_EAGAIN;
    }
    // the memory may have been used by anyone since the last call: carve it
    // for exactly these sizes and clear the arena
    sV = std::max<int64_t>(sV, 2);
    sE = std::max<int64_t>(sE, 1);
    sn = std::max<int32_t>(sn, 1);
    const size_t abytes = arena_bytes(Vcap, Mcap, Ecap, ncap), sbytes = scratch_bytes(sV, sE, sn);
    if (abytes + sbytes > ext_bytes_) {
      char buf[200];
      std::snprintf(buf, sizeof(buf),
                    "the graph needs %zu bytes of device memory (arena %zu + builder %zu), more than the %zu bytes "
                    "of the allocation-free entry point",
                    abytes + sbytes, abytes, sbytes, ext_bytes_);
      *err = buf;
      return WBPR_ETOOBIG;
    }
    drop_graphs();
    arena_ = ext_base_;
    arena_n_ = abytes;
    scratch_ = (char *)ext_base_ + abytes;  // abytes is a multiple of 256
    scratch_n_ = sbytes;
    sV_ = sV;
    sE_ = sE;
    sn_ = sn;
    carve(Vcap, Mcap, Ecap, ncap);
    hipError_t e = hipMemset(arena_, 0, abytes);
    if (e == hipSuccess) e = hipMemset(inst_of_, 0xff, 4 * (size_t)Vcap);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      *err = std::string("arena init: ") + hipGetErrorString(e);
      return WBPR_EDEVICE;
    }
    reset_books();
    e = ensure_pinned(err);
    return e == hipSuccess ? 0 : WBPR_ENOMEM;
  }
  const bool grow_arena = Vcap > Vcap_ || Mcap > Mcap_ || Ecap > Ecap_ || ncap > ncap_;
  if (grow_arena && resident_ > 0) {
    *err = "arena cannot grow while instances are resident";
    return WBPR_EAGAIN;
  }
  if (grow_arena) {
    drop_graphs();
    Vcap = std::max(Vcap, Vcap_);
    Mcap = std::max(Mcap, Mcap_);
    Ecap = std::max(Ecap, Ecap_);
    ncap = std::max(ncap, ncap_);
    const size_t bytes = arena_bytes(Vcap, Mcap, Ecap, ncap);
    if (arena_) hipFree(arena_);
    arena_ = nullptr;
    arena_n_ = 0;
    hipError_t e = hipMalloc(&arena_, bytes);
    if (e != hipSuccess) {
      *err = std::string("arena allocation: ") + hipGetErrorString(e);
      Vcap_ = Mcap_ = Ecap_ = 0;
      ncap_ = 0;
      return e == hipErrorOutOfMemory ? WBPR_ENOMEM : WBPR_EDEVICE;
    }
    arena_n_ = bytes;
    carve(Vcap, Mcap, Ecap, ncap);
    // free arena: empty rows, inactive vertices, no instance
    e = hipMemset(arena_, 0, bytes);
    if (e == hipSuccess) e = hipMemset(inst_of_, 0xff, 4 * (size_t)Vcap);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      *err = std::string("arena init: ") + hipGetErrorString(e);
      return WBPR_EDEVICE;
    }
    reset_books();
    e = ensure_pinned(err);
    if (e != hipSuccess) return WBPR_ENOMEM;
  }
  sV_ = std::max(sV_, sV);
  sE_ = std::max(sE_, sE);
  sn_ = std::max(sn_, sn);
  const size_t sbytes = scratch_bytes(sV_, sE_, sn_);
  if (sbytes > scratch_n_) {
    if (resident_ > 0 && scratch_) hipDeviceSynchronize();
    if (scratch_) hipFree(scratch_);
    scratch_ = nullptr;
    scratch_n_ = 0;
    hipError_t e = hipMalloc(&scratch_, sbytes);
    if (e != hipSuccess) {
      *err = std::string("scratch allocation: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? WBPR_ENOMEM : WBPR_EDEVICE;
    }
    scratch_n_ = sbytes;
  }
  return 0;
}

// Points every arena array into arena_ (arena_bytes(...) long).
void Engine::carve(int64_t Vcap, int64_t Mcap, int64_t Ecap, int32_t ncap) {
  gr_uploaded_.clear();
  {
    Vcap_ = Vcap;
    Mcap_ = Mcap;
    Ecap_ = Ecap;
    ncap_ = ncap;
    char *p = (char *)arena_;
    auto take = [&](size_t n) { char *q = p; p += al(n); return (void *)q; };
    A_.rowb = (int2 *)take(8 * (size_t)Vcap);
    A_.ent = (int2 *)take(8 * (size_t)Mcap);
    A_.rev = (int32_t *)take(4 * (size_t)Mcap);
    A_.cap0 = (int32_t *)take(4 * (size_t)Mcap);
    A_.arc2ent = (int32_t *)take(4 * (size_t)Ecap);
    A_.pbefore = (int32_t *)take(4 * (size_t)Ecap);
    A_.acap = (int32_t *)take(4 * (size_t)Ecap);
    e_ = (long long *)take(8 * (size_t)Vcap);
    h_ = (int32_t *)take(4 * (size_t)Vcap);
    inst_of_ = (int32_t *)take(4 * (size_t)Vcap);
    q_[0] = (int32_t *)take(4 * (size_t)Vcap);
    q_[1] = (int32_t *)take(4 * (size_t)Vcap);
    mid_ = (int32_t *)take(4 * (size_t)mid_words(Vcap));
    fq_[0] = (int32_t *)take(4 * (size_t)Vcap);
    fq_[1] = (int32_t *)take(4 * (size_t)Vcap);
    big_ = (int32_t *)take(4 * (size_t)Vcap);
    lr_cnt_ = (int32_t *)take(4 * (size_t)Vcap);
    tcap_ = task_capacity(Vcap, Mcap);
    task_u_ = (int32_t *)take(4 * (size_t)tcap_);
    task_c_ = (int32_t *)take(4 * (size_t)tcap_);
    vis_ = (uint8_t *)take((size_t)Vcap);
    gap_hist_ = (int32_t *)take(4 * (size_t)GAP_BINS);
    nchunk_ = chunk_capacity(Vcap, Mcap, chunk_);
    chunk_w_ = (int32_t *)take(8 * (size_t)nchunk_);
    chunk_b_ = chunk_w_ + nchunk_;
    // the BFS chunk descriptors are idle during sweeps: the long rows'
    // minimum keys live there
    lr_key_ = reinterpret_cast<unsigned long long *>(chunk_w_);
    inst_active_ = (int32_t *)take(4 * (size_t)ncap);
    inst_stranded_ = (int32_t *)take(4 * (size_t)ncap);
    roots_ = (int32_t *)take(4 * (size_t)ncap);
    root_h_ = (int32_t *)take(4 * (size_t)ncap);
    excl_ = (int32_t *)take(4 * (size_t)ncap);
    dbg_term_ = (int2 *)take(8 * (size_t)ncap);
    inst_list_ = take(sizeof(InstDev) * (size_t)ncap * kListKinds + 4 * (size_t)ncap);
    pk_ring_ = (WgInst *)take(sizeof(WgInst) * (size_t)ncap);
    pk_stage_ = (WgInst *)take(sizeof(WgInst) * (size_t)ncap);
    pk_result_ = (int32_t *)take(4 * (size_t)ncap);
    misc_ = (long long *)take(sizeof(MiscLayout));
    sweep_log_dev_ = (int32_t *)take(6 * 4 * (size_t)kSweepLogCap);
    sweep_log_ = log_level() >= 2 ? sweep_log_dev_ : nullptr;
    MiscLayout *m = reinterpret_cast<MiscLayout *>(misc_);
    sink_ = &m->sink;
    budget_ = &m->budget;
  }
}

// Host bookkeeping of an empty arena.
void Engine::reset_books() {
  valloc_.reset(Vcap_);
  malloc_.reset(Mcap_);
  aalloc_.reset(Ecap_);
  slot_free_.clear();
  for (int32_t i = ncap_ - 1; i >= 0; i--) slot_free_.push_back(i);
  inst_.assign(ncap_, Inst());
  groups_.clear();
  resident_ = 0;
  resident_V_ = 0;
  resident_M_ = 0;
}

// Pinned host staging for the instance lists and read-backs.
hipError_t Engine::ensure_pinned(std::string *err) {
  const size_t pin_need = kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds + 24 * (size_t)ncap_ + 4096;
  if (pin_n_ >= pin_need) return hipSuccess;
  if (external_) {  // plain host memory: no HIP allocation
    ext_host_.assign(pin_need, 0);
    pin_ = ext_host_.data();
    pin_n_ = pin_need;
    return hipSuccess;
  }
  if (pin_) hipHostFree(pin_);
  pin_ = nullptr;
  pin_n_ = 0;
  hipError_t e = hipHostMalloc((void **)&pin_, pin_need, hipHostMallocDefault);
  if (e != hipSuccess) {
    *err = std::string("pinned staging: ") + hipGetErrorString(e);
    return e;
  }
  pin_n_ = pin_need;
  return hipSuccess;
}

// Longest row each listed instance's sweeps can meet (terminals excluded),
// stored in its Inst.  Synchronises the stream.
int Engine::measure_rows(const std::vector<int> &slots, hipStream_t st, std::string *err) {
  if (slots.empty()) return 0;
  hipError_t e = hipMemsetAsync(inst_stranded_, 0, 4 * slots.size(), st);
  if (e != hipSuccess) {
    *err = std::string("row measure: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  launch_inst_kernel(IK_MAXDEG, slots, st);
  int32_t *h = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                           16 * (size_t)ncap_);
  e = hipMemcpyAsync(h, inst_stranded_, 4 * slots.size(), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = std::string("row measure: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  for (size_t i = 0; i < slots.size(); i++) inst_[slots[i]].maxdeg = h[i];
  return 0;
}

void Engine::launch_inst_kernel(int which, const std::vector<int> &slots, hipStream_t st) {
  std::vector<InstDev> list;
  list.reserve(slots.size());
  for (int sl : slots) {
    const Inst &I = inst_[sl];
    InstDev d;
    d.vbase = I.vbase;
    d.V = I.V;
    d.s = I.s;
    d.t = I.t;
    d.abase = I.abase;
    d.E = I.E;
    d.value = (long long *)I.value;
    d.flow = I.flow;
    d.side = I.side;
    list.push_back(d);
  }
  launch_inst_list(which, list, slots, st);
}

// Per-instance kernel over a list of descriptors.  Each kernel kind has its
// own pinned and device staging slice; a slice is reused only after the
// stream has been synchronised (every round and every admission syncs).
void Engine::launch_inst_list(int which, const std::vector<InstDev> &list, const std::vector<int> &slots,
                              hipStream_t st) {
  const int n = (int)list.size();
  if (n == 0) return;
  InstDev *hl = reinterpret_cast<InstDev *>(pin_ + kPinnedHeader) + (size_t)which * ncap_;
  InstDev *dl = reinterpret_cast<InstDev *>(inst_list_) + (size_t)which * ncap_;
  int32_t *dslot = reinterpret_cast<int32_t *>(reinterpret_cast<InstDev *>(inst_list_) + (size_t)kListKinds * ncap_);
  int32_t *hslot = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds);
  int64_t maxlen = 1;
  for (int i = 0; i < n; i++) {
    hl[i] = list[i];
    if (which == IK_INIT) hslot[i] = slots[i];
    maxlen = std::max<int64_t>(maxlen, which == IK_DECODE ? list[i].E : list[i].V);
  }
  hipMemcpyAsync(dl, hl, sizeof(InstDev) * n, hipMemcpyHostToDevice, st);
  if (which == IK_INIT) hipMemcpyAsync(dslot, hslot, 4 * (size_t)n, hipMemcpyHostToDevice, st);
  InstArgs a{dl, A_.rowb, A_.ent, A_.rev, A_.cap0, A_.arc2ent, A_.pbefore, A_.acap, e_, h_, inst_of_, dslot,
             inst_stranded_, cfg_.rcsr ? 1 : 0};
  // the decode's per-arc chain of dependent gathers wants every wave slot
  unsigned bx = which == IK_VALUE_ZERO || which == IK_PHASE2 ? 1u : grid1d(maxlen, 256, which == IK_DECODE ? 4096 : 1024);
  if (which == IK_PREFLOW || which == IK_VALUE) bx = 64;
  for (int off = 0; off < n; off += 65535) {
    const int cnt = std::min(65535, n - off);
    InstArgs b = a;
    b.L = dl + off;
    b.slot = dslot + off;
    b.maxdeg = a.maxdeg + off;
    hipLaunchKernelGGL(k_inst, dim3(bx, cnt), dim3(256), 0, st, b, which);
  }
}

// The largest LDS a workgroup of the small-instance kernel may have, less
// the static part (once; -1 when the device cannot give enough).
void Engine::prime_small_lds() {
  if (small_lds_ != 0) return;
  int dev_max = 0;
  if (hipDeviceGetAttribute(&dev_max, hipDeviceAttributeMaxSharedMemoryPerBlock, device_) != hipSuccess ||
      dev_max - 2048 < 32768 ||
      hipFuncSetAttribute((const void *)k_small_solve, hipFuncAttributeMaxDynamicSharedMemorySize, dev_max - 2048) !=
          hipSuccess) {
    hipGetLastError();
    small_lds_ = -1;  // no LDS-resident path on this device
    return;
  }
  small_lds_ = dev_max - 2048;
}

// A freshly started group of small instances, alone on the device, is
// solved whole: one workgroup per instance with its residual graph in LDS;
// the instances are then retired by the next round like any finished one
// (those that do not fit the LDS budget stay with the rounds, untouched).
// Not when other instances are resident or the group holds a larger one:
// there the small instances ride along in the shared rounds for little, and
// a solve at admission would hold up everything else (measured: batched
// solves/s 15.6k -> 12.4k, served p50 6.3 -> 9.4 ms).
int Engine::solve_small(const std::vector<int> &slots, hipStream_t st, std::string *err) {
  // BCSR only: the LDS copy of a row keeps 16-bit mates
  if (cfg_.rcsr || cfg_.debug_checks || cfg_.lds_max_v < 0 || small_lds_ < 0 || resident_ != (int)slots.size())
    return 0;
  const int vmax = cfg_.lds_max_v > 0 ? cfg_.lds_max_v : 1024;
  std::vector<int> cand;
  for (int sl : slots)
    if (inst_[sl].V <= vmax) cand.push_back(sl);
  if (cand.empty() || cand.size() != slots.size()) return 0;
  prime_small_lds();
  if (small_lds_ < 0) return 0;
  const int n = (int)cand.size();
  InstDev *hl = reinterpret_cast<InstDev *>(pin_ + kPinnedHeader) + (size_t)IK_SMALL * ncap_;
  InstDev *dl = reinterpret_cast<InstDev *>(inst_list_) + (size_t)IK_SMALL * ncap_;
  for (int i = 0; i < n; i++) {
    const Inst &I = inst_[cand[i]];
    InstDev d;
    d.vbase = I.vbase;
    d.V = I.V;
    d.s = I.s;
    d.t = I.t;
    d.abase = I.abase;
    d.E = I.E;
    d.value = (long long *)I.value;
    d.flow = I.flow;
    d.side = I.side;
    hl[i] = d;
  }
  hipError_t e = hipMemcpyAsync(dl, hl, sizeof(InstDev) * n, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) {
    *err = std::string("small solve: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  // WBPR_LDS_ROUND_CAP (tests only) lowers the round cap so that the
  // hand-over of an unfinished instance to the rounds can be exercised
  const char *cap_env = std::getenv("WBPR_LDS_ROUND_CAP");
  const int32_t round_cap = cap_env ? std::max(0, std::atoi(cap_env)) : 0;
  SmallArgs sa{dl, A_.rowb, A_.ent, A_.rev, A_.cap0, e_, h_, inst_stranded_, misc->stats, small_lds_, round_cap};
  hipLaunchKernelGGL(k_small_solve, dim3(n), dim3(SMALL_THREADS), small_lds_, st, sa);
  int32_t *hres = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                              8 * (size_t)ncap_);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hres, inst_stranded_, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = std::string("small solve: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  std::vector<int> solved, decode;
  for (int i = 0; i < n; i++) {
    // an instance that reached the round cap wrote nothing back: it is still
    // in its preflow state and the rounds of launches solve it
    if (hres[i] == 2) acc_.small_fallbacks++;
    if (hres[i] != 1) continue;
    Inst &I = inst_[cand[i]];
    solved.push_back(cand[i]);
    if (I.flow) decode.push_back(cand[i]);
    I.phase = 3;
    I.pending_done = true;
  }
  launch_inst_kernel(IK_DECODE, decode, st);
  acc_.small_solved += (int64_t)solved.size();
  return 0;
}

// Instances eligible for the persistent workgroup-per-instance kernel
// (batch_kernel = 2): up to WG_MAX_V vertices and WG_MAX_E arcs, in a group
// alone on the device (a kernel at admission would hold up instances
// already in the rounds).
constexpr int32_t WG_MAX_V = 1 << 17;
constexpr int64_t WG_MAX_E = 1 << 20;
// An instance still unsolved after this long in the persistent kernel is
// handed to the rounds (a safety limit: the largest eligible instances take
// a few hundred milliseconds in one workgroup).
constexpr double kWgMaxMs = 2000.0;

// Descriptor of instance I for the persistent kernel, with its schedule:
// tile width by its row lengths (as the rounds choose it), relabel budget
// from the options.
void Engine::fill_wg(const Inst &I, WgInst *d) const {
  d->vbase = I.vbase;
  d->V = I.V;
  d->s = I.s;
  d->t = I.t;
  d->abase = I.abase;
  d->E = I.E;
  d->value = (long long *)I.value;
  d->flow = I.flow;
  d->side = I.side;
  const double mean_row = I.V > 0 ? 2.0 * (double)I.E / (double)I.V : 1.0;
  d->lanes = cfg_.lanes_per_vertex > 0 ? cfg_.lanes_per_vertex
             : I.maxdeg <= 16          ? 1
             : mean_row <= 10.0        ? 4
             : mean_row <= 20.0        ? 8
                                       : 16;
  d->budget_pm = cfg_.gr_work_permille;
}

int Engine::solve_wg(const std::vector<int> &slots, hipStream_t st, std::string *err) {
  // only on request (batch_kernel = 2): one workgroup per instance measured
  // slower than the shared rounds for every size the LDS-resident solve
  // does not take (instances above 1,024 vertices) and 3.6 times slower on
  // the batched stream's mix of sizes
  if (cfg_.batch_kernel != 2 || cfg_.debug_checks || resident_ != (int)slots.size()) return 0;
  std::vector<int> cand;
  for (int sl : slots) {
    const Inst &I = inst_[sl];
    if (I.phase == 1 && !I.pending_done && I.V <= WG_MAX_V && I.E <= WG_MAX_E) cand.push_back(sl);
  }
  if (cand.empty()) return 0;
  // largest first: the longest solves start first, the rest fill in behind
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return inst_[a].E > inst_[b].E; });
  const int n = (int)cand.size();
  WgInst *hl = reinterpret_cast<WgInst *>(reinterpret_cast<InstDev *>(pin_ + kPinnedHeader) + (size_t)IK_WG * ncap_);
  WgInst *dl = reinterpret_cast<WgInst *>(reinterpret_cast<InstDev *>(inst_list_) + (size_t)IK_WG * ncap_);
  static_assert(sizeof(WgInst) <= sizeof(InstDev), "WgInst must fit its list slice");
  for (int i = 0; i < n; i++) fill_wg(inst_[cand[i]], &hl[i]);
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  hipError_t e = hipMemcpyAsync(dl, hl, sizeof(WgInst) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(misc->wg_head, 0, sizeof(misc->wg_head), st);
  if (e == hipSuccess) e = hipMemsetAsync(inst_stranded_, 0, 4 * (size_t)n, st);
  if (e != hipSuccess) {
    *err = std::string("persistent batch: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  WgArgs a{};
  a.L = dl;
  a.n = n;
  a.head = misc->wg_head;
  a.tail = nullptr;
  a.close = nullptr;
  a.idle_ticks = 0;
  a.result = inst_stranded_;
  a.rowb = A_.rowb;
  a.ent = A_.ent;
  a.rev = A_.rev;
  a.cap0 = A_.cap0;
  a.arc2ent = A_.arc2ent;
  a.pbefore = A_.pbefore;
  a.acap = A_.acap;
  a.e = e_;
  a.h = h_;
  a.qa = q_[0];
  a.qb = q_[1];
  a.stats = misc->wg_stats;
  // WBPR_WG_ROUND_CAP (tests only) lowers the round cap so that the
  // hand-over of unfinished instances to the rounds can be exercised
  const char *cap_env = std::getenv("WBPR_WG_ROUND_CAP");
  a.round_cap = cap_env ? std::max(0, std::atoi(cap_env)) : 0;
  a.max_ticks = (long long)(kWgMaxMs * 1e5);  // 100 MHz device clock
  launch_wg_solve(cfg_.rcsr, std::min(n, 2048), st, a);
  int32_t *hres = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                              8 * (size_t)ncap_);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(hres, inst_stranded_, 4 * (size_t)n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = std::string("persistent batch: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  for (int i = 0; i < n; i++) {
    Inst &I = inst_[cand[i]];
    if (hres[i] == 1) {  // solved, flows decoded
      I.phase = 3;
      I.pending_done = true;
      acc_.wg_solved++;
    } else if (hres[i] == 2 || hres[i] == 3) {  // stopped at a cap: the rounds finish it
      if (hres[i] == 3) I.phase = 2;  // value and side written, s carries its phase-2 bias
      acc_.wg_fallbacks++;
    } else {
      *err = "persistent batch: an instance was not processed";
      return WBPR_EINTERNAL;
    }
  }
  return 0;
}

int Engine::admit(const GroupInput &in, hipStream_t st, std::string *err) {
  if (in.n <= 0) return 0;
  if (in.keep && in.n != 1) {
    *err = "only single-instance groups can be kept";
    return WBPR_EINVAL;
  }
  if (in.start && in.n > (int32_t)slot_free_.size()) {
    *err = "no free instance slot";
    return WBPR_EAGAIN;
  }
  int64_t Vt = 0, Et = 0;
  for (int i = 0; i < in.n; i++) {
    Vt += in.V[i];
    Et += in.E[i];
  }
  if (Vt >= (1ll << 30) || 2 * Et >= (1ll << 31) - 1) {
    *err = "group exceeds the 32-bit index limits";
    return WBPR_ETOOBIG;
  }
  if (Vt > sV_ || Et > sE_ || in.n > sn_) {
    int rc = reserve(0, 0, 0, 0, Vt, Et, in.n, err);
    if (rc) return rc;
  }
  const int64_t vb = valloc_.alloc(Vt);
  const int64_t mb = vb < 0 ? -1 : malloc_.alloc(std::max<int64_t>(2 * Et, 1));
  const int64_t ab = mb < 0 ? -1 : aalloc_.alloc(std::max<int64_t>(Et, 1));
  if (vb < 0 || mb < 0 || ab < 0) {
    if (vb >= 0) valloc_.release(vb, Vt);
    if (mb >= 0) malloc_.release(mb, std::max<int64_t>(2 * Et, 1));
    *err = "arena full";
    return WBPR_EAGAIN;
  }
  // scratch carve: builder | union rows | union cols | voff | eoff | bad | status
  char *sp = (char *)scratch_;
  void *bscratch = sp;
  sp += al(build_scratch_bytes((int32_t)sV_, sE_));
  int64_t *rp_union = (int64_t *)sp;
  sp += al(8 * ((size_t)sV_ + 1));
  int32_t *col_union = (int32_t *)sp;
  sp += al(4 * (size_t)(sE_ > 0 ? sE_ : 1));
  int32_t *voff = (int32_t *)sp;
  sp += al(4 * ((size_t)sn_ + 1));
  int64_t *eoff = (int64_t *)sp;
  sp += al(8 * ((size_t)sn_ + 1));
  int32_t *bad = (int32_t *)sp;
  sp += al(4 * (size_t)sn_);
  BuildStatus *bst = (BuildStatus *)sp;

  const int64_t *rp = in.row_ptr;
  const int32_t *col = in.col;
  if (in.n > 1) {
    // prefix offsets of the instances (host) -> device
    std::vector<int32_t> voh(in.n + 1);
    std::vector<int64_t> eoh(in.n + 1);
    voh[0] = 0;
    eoh[0] = 0;
    for (int i = 0; i < in.n; i++) {
      voh[i + 1] = voh[i] + in.V[i];
      eoh[i + 1] = eoh[i] + in.E[i];
    }
    // the offsets are small; a synchronised copy keeps the staging simple
    hipError_t e = hipMemcpyAsync(voff, voh.data(), 4 * (size_t)(in.n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(eoff, eoh.data(), 8 * (size_t)(in.n + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(bad, 0, 4 * (size_t)in.n, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // pageable sources
    if (e != hipSuccess) {
      valloc_.release(vb, Vt);
      malloc_.release(mb, std::max<int64_t>(2 * Et, 1));
      aalloc_.release(ab, std::max<int64_t>(Et, 1));
      *err = std::string("group offsets: ") + hipGetErrorString(e);
      return WBPR_EDEVICE;
    }
    hipLaunchKernelGGL(k_union_rows, dim3(grid1d(Vt + 1)), dim3(256), 0, st, in.n, voff, eoff, in.row_ptr, rp_union,
                       bad);
    if (Et > 0)
      hipLaunchKernelGGL(k_union_cols, dim3(grid1d(Et)), dim3(256), 0, st, in.n, voff, eoff, in.col, col_union, bad);
    rp = rp_union;
    col = col_union;
  }
  Place pl;
  pl.vbase = (int32_t)vb;
  pl.mbase = mb;
  pl.abase = ab;
  int evb = -1;
  if (cfg_.time_kernels) {  // the builder's device time (events on the stream)
    if (ev_used_ + 2 > (int)ev_.size()) {
      const size_t old = ev_.size();
      ev_.resize(old + 1024);
      for (size_t i = old; i < ev_.size(); i++) hipEventCreate(&ev_[i]);
    }
    evb = ev_used_;
    ev_used_ += 2;
    ev_marks_.push_back({5, evb});
    hipEventRecord(ev_[evb], st);
  }
  hipError_t e = cfg_.rcsr ? build_residual_rcsr(rp, col, in.cap, (int32_t)Vt, Et, A_, pl, bscratch, bst, st)
                           : build_residual(rp, col, in.cap, (int32_t)Vt, Et, A_, pl, bscratch, bst, st);
  if (evb >= 0 && e == hipSuccess) e = hipEventRecord(ev_[evb + 1], st);
  BuildStatus hb;
  if (e == hipSuccess) e = hipMemcpyAsync(pin_, bst, sizeof(BuildStatus), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  int bad_any = 0;
  if (e == hipSuccess) {
    std::memcpy(&hb, pin_, sizeof(hb));
    if (in.n > 1) {
      std::vector<int32_t> hbad(in.n);
      hipError_t e2 = hipMemcpy(hbad.data(), bad, 4 * (size_t)in.n, hipMemcpyDeviceToHost);
      if (e2 != hipSuccess) e = e2;
      for (int i = 0; i < in.n && e == hipSuccess; i++) bad_any |= hbad[i] != 0;
    }
  }
  auto undo = [&]() {
    valloc_.release(vb, Vt);
    malloc_.release(mb, std::max<int64_t>(2 * Et, 1));
    aalloc_.release(ab, std::max<int64_t>(Et, 1));
  };
  if (e != hipSuccess) {
    undo();
    *err = std::string("residual build: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  if (hb.bad_input || bad_any || hb.overflow) {
    // empty the rows written for this group before its ranges are reused
    hipMemsetAsync(A_.rowb + vb, 0, 8 * (size_t)Vt, st);
    hipStreamSynchronize(st);
    undo();
    if (hb.overflow && !hb.bad_input && !bad_any) {
      *err = "c(u->v) + c(v->u) over parallel arcs exceeds INT32_MAX";
      return WBPR_EOVERFLOW;
    }
    *err = "malformed CSR (row_ptr not monotone from 0 to E, col out of range, or negative cap)";
    return WBPR_EINVAL;
  }
  const int64_t Mres = std::max<int64_t>(2 * Et, 1);
  malloc_.shrink(mb, Mres, std::max<int64_t>(hb.M, 1));
  last_M_ = hb.M;
  // register the group and its instances
  int gi = -1;
  for (int i = 0; i < (int)groups_.size(); i++)
    if (!groups_[i].used) {
      gi = i;
      break;
    }
  if (gi < 0) {
    groups_.push_back(Group());
    gi = (int)groups_.size() - 1;
  }
  Group &G = groups_[gi];
  G.used = true;
  G.tag = in.tag;
  G.vbase = (int32_t)vb;
  G.V = (int32_t)Vt;
  G.mbase = mb;
  G.Mres = std::max<int64_t>(hb.M, 1);
  G.abase = ab;
  G.E = Et;
  G.keep = in.keep;
  if (in.group_out) *in.group_out = gi;
  resident_V_ += Vt;
  resident_M_ += hb.M;
  if (!in.start) {  // built only: instances start later
    G.remaining = 0;
    return 0;
  }
  G.remaining = in.n;
  std::vector<int> slots(in.n);
  int64_t vo = 0, eo = 0;
  for (int i = 0; i < in.n; i++) {
    const int sl = slot_free_.back();
    slot_free_.pop_back();
    slots[i] = sl;
    Inst &I = inst_[sl];
    I.used = true;
    I.V = in.V[i];
    I.E = in.E[i];
    I.vbase = (int32_t)(vb + vo);
    I.s = I.vbase + in.s[i];
    I.t = I.vbase + in.t[i];
    I.abase = ab + eo;
    I.phase = 1;
    I.group = gi;
    I.index = i;
    I.value = in.values ? in.values + i : nullptr;
    I.flow = in.flows ? in.flows + eo : nullptr;
    I.side = in.sides ? in.sides + vo : nullptr;
    vo += in.V[i];
    eo += in.E[i];
  }
  resident_ += in.n;
  launch_inst_kernel(IK_INIT, slots, st);
  launch_inst_kernel(IK_PREFLOW, slots, st);
  int rc = measure_rows(slots, st, err);
  if (rc) return rc;
  if (in.persistent) {
    rc = pk_publish(slots, st, err);
    if (rc) return rc;
  } else {
    rc = solve_small(slots, st, err);
    if (rc) return rc;
    rc = solve_wg(slots, st, err);
    if (rc) return rc;
  }
  e = hipGetLastError();
  if (e != hipSuccess) {
    *err = std::string("instance init: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  return 0;
}

// Invariants of a preflow (section 2.2) on a state with no sweep running,
// for the vertices of the instances whose slot has terminals term[slot] =
// {s, t} (x = -1: not checked; option debug_checks): no residual is
// negative; BCSR: an entry's and its mate's residuals sum to the pair's
// merged capacities; RCSR: a forward entry's residual plus its arc's flow is
// the arc's capacity, the flow not negative; every vertex other than s and t
// holds exactly its inflow minus its outflow over its row, and not less than
// 0.  One wave per vertex; bad[0] counts entries, bad[1] vertices.
__global__ void __launch_bounds__(256) k_debug_check(const int2 *rowb, const int2 *ent, const int32_t *rev,
                                                     const int32_t *cap0, const long long *e, const int32_t *inst_of,
                                                     const int2 *term, int32_t nv, int rcsr,
                                                     unsigned long long *bad) {
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WB_WAVE;
  long long bad_ent = 0, bad_vtx = 0;
  for (int64_t v = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WB_WAVE; v < nv; v += nw) {  // wave-uniform
    const int32_t sl = inst_of[v];
    if (sl < 0) continue;
    const int2 st = term[sl];
    if (st.x < 0) continue;
    const int2 rb = rowb[v];
    long long inflow = 0;  // inflow minus outflow
    for (int32_t k = rb.x + lane(); k < rb.y; k += WB_WAVE) {
      const int2 cr = ent[k];
      if (!rcsr) {
        const int32_t m = rev[k];
        if (cr.y < 0 || (long long)cr.y + ent[m].y != (long long)cap0[k] + cap0[m]) bad_ent++;
        inflow += (long long)cr.y - cap0[k];
      } else if (cr.x >= 0) {
        const int32_t f = rev[k];
        if (cr.y < 0 || f < 0 || (long long)cr.y + f != (long long)cap0[k]) bad_ent++;
        inflow -= f;
      } else {
        inflow += rev[cr.y];
      }
    }
    inflow = group_sum_i64<WB_WAVE>(inflow);
    const long long ev = e[v];
    if (lane() == 0 && v != st.x && v != st.y && (ev < 0 || ev != inflow)) bad_vtx++;
  }
  bad_ent = group_sum_i64<WB_WAVE>(bad_ent);
  bad_vtx = group_sum_i64<WB_WAVE>(bad_vtx);
  if (lane() == 0 && bad_ent) atomicAdd(&bad[0], (unsigned long long)bad_ent);
  if (lane() == 0 && bad_vtx) atomicAdd(&bad[1], (unsigned long long)bad_vtx);
}

int Engine::debug_check(hipStream_t st, int32_t vhi, std::string *err) {
  std::vector<int2> term(ncap_, make_int2(-1, -1));
  for (int i = 0; i < ncap_; i++)
    if (inst_[i].used && (inst_[i].phase == 1 || inst_[i].phase == 2)) term[i] = make_int2(inst_[i].s, inst_[i].t);
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  unsigned long long hb[2] = {0, 0};
  hipError_t e = hipSuccess;
  // WBPR_DEBUG_PLANT (tests only): before the first check, the host adds one
  // unit of excess to a vertex other than s and t, a conservation violation
  // the check must report
  if (acc_.debug_checked == 0 && std::getenv("WBPR_DEBUG_PLANT")) {
    for (int i = 0; i < ncap_; i++) {
      const Inst &I = inst_[i];
      if (term[i].x < 0 || I.V < 3) continue;
      int32_t v = I.vbase;
      while (v == I.s || v == I.t) v++;
      long long x = 0;
      e = hipMemcpyAsync(&x, e_ + v, 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      x += 1;
      if (e == hipSuccess) e = hipMemcpyAsync(e_ + v, &x, 8, hipMemcpyHostToDevice, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      break;
    }
  }
  if (e == hipSuccess) e = hipMemcpyAsync(dbg_term_, term.data(), 8 * (size_t)ncap_, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemsetAsync(misc->dbg, 0, sizeof(misc->dbg), st);
  if (e == hipSuccess) {
    const int64_t waves = std::max<int64_t>(vhi, 1);
    hipLaunchKernelGGL(k_debug_check, dim3(grid1d(waves * WB_WAVE, 256, 16384)), dim3(256), 0, st, A_.rowb, A_.ent,
                       A_.rev, A_.cap0, e_, inst_of_, dbg_term_, vhi, cfg_.rcsr ? 1 : 0, misc->dbg);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hb, misc->dbg, sizeof(hb), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = std::string("debug check: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  if (hb[0] || hb[1]) {
    char buf[160];
    std::snprintf(buf, sizeof(buf),
                  "debug check before global relabel %lld: %llu entries and %llu vertices violate the preflow "
                  "invariants",
                  (long long)acc_.global_relabels + 1, hb[0], hb[1]);
    *err = buf;
    return WBPR_EINTERNAL;
  }
  acc_.debug_checked++;
  return 0;
}

// Residuals back to the input capacities; RCSR also zeroes every arc's flow
// (reverse entries hold an index, not a residual, and stay as they are).
__global__ void k_reset_entries(int2 *ent, const int32_t *cap0, int32_t *flow, int rcsr, int64_t M) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M; k += (int64_t)gridDim.x * blockDim.x) {
    if (!rcsr) {
      ent[k].y = cap0[k];
    } else if (ent[k].x >= 0) {
      ent[k].y = cap0[k];
      flow[k] = 0;
    }
  }
}

bool Engine::has_kept_groups() const {
  for (const Group &G : groups_)
    if (G.used && G.keep) return true;
  return false;
}

int Engine::start_instance(int gid, int32_t s, int32_t t, int64_t *value, int32_t *flow, uint8_t *side, uint64_t tag,
                           hipStream_t st, std::string *err) {
  if (gid < 0 || gid >= (int)groups_.size() || !groups_[gid].used || !groups_[gid].keep) {
    *err = "no such kept graph";
    return WBPR_EINVAL;
  }
  Group &G = groups_[gid];
  if (G.remaining != 0) {
    *err = "the graph is being solved";
    return WBPR_EAGAIN;
  }
  if (s < 0 || s >= G.V || t < 0 || t >= G.V || s == t) {
    *err = "s or t out of range, or s == t";
    return WBPR_EINVAL;
  }
  if (slot_free_.empty()) {
    *err = "no free instance slot";
    return WBPR_EAGAIN;
  }
  // residual capacities back to the merged input capacities
  hipLaunchKernelGGL(k_reset_entries, dim3(grid1d(G.Mres, 256, 16384)), dim3(256), 0, st, A_.ent + G.mbase,
                     A_.cap0 + G.mbase, A_.rev + G.mbase, cfg_.rcsr ? 1 : 0, G.Mres);
  const int sl = slot_free_.back();
  slot_free_.pop_back();
  Inst &I = inst_[sl];
  I = Inst();
  I.used = true;
  I.V = G.V;
  I.E = G.E;
  I.vbase = G.vbase;
  I.s = G.vbase + s;
  I.t = G.vbase + t;
  I.abase = G.abase;
  I.phase = 1;
  I.group = gid;
  I.index = 0;
  I.value = value;
  I.flow = flow;
  I.side = side;
  G.tag = tag;
  G.remaining = 1;
  resident_ += 1;
  launch_inst_kernel(IK_INIT, std::vector<int>{sl}, st);
  launch_inst_kernel(IK_PREFLOW, std::vector<int>{sl}, st);
  int rc = measure_rows(std::vector<int>{sl}, st, err);
  if (rc) return rc;
  rc = solve_small(std::vector<int>{sl}, st, err);
  if (rc) return rc;
  rc = solve_wg(std::vector<int>{sl}, st, err);
  if (rc) return rc;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    *err = std::string("instance init: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  return 0;
}

void Engine::free_group(int gid, hipStream_t st) {
  if (gid < 0 || gid >= (int)groups_.size() || !groups_[gid].used || groups_[gid].remaining != 0) return;
  groups_[gid].keep = false;
  release_groups(std::vector<int>{gid}, st);
}

// Clears the vertices of the listed groups (rows, excess, heights, owner)
// in one launch, then returns their ranges.  One launch per call: the pinned
// descriptor slice of a kernel kind is rewritten only after a stream sync.
void Engine::release_groups(const std::vector<int> &gis, hipStream_t st) {
  if (gis.empty()) return;
  std::vector<InstDev> list;
  for (int gi : gis) {
    Group &G = groups_[gi];
    InstDev d;
    std::memset(&d, 0, sizeof(d));
    d.vbase = G.vbase;
    d.V = G.V;
    list.push_back(d);
  }
  launch_inst_list(IK_RELEASE, list, std::vector<int>(list.size(), 0), st);
  for (int gi : gis) {
    Group &G = groups_[gi];
    valloc_.release(G.vbase, G.V);
    malloc_.release(G.mbase, G.Mres);
    aalloc_.release(G.abase, std::max<int64_t>(G.E, 1));
    resident_V_ -= G.V;
    resident_M_ -= G.Mres;
    G.used = false;
  }
}

// Captured batch of K sweeps (one cached graph per K).
int Engine::ensure_graph(hipStream_t st, int K, int tiers, hipGraphExec_t *exec, std::string *err) {
  const int key = 4 * K + tiers;
  auto it = graphs_.find(key);
  if (it != graphs_.end()) {
    *exec = it->second.second;
    return 0;
  }
  hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    *err = std::string("graph capture: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  enqueue_sweeps(st, K, tiers);
  hipGraph_t graph = nullptr;
  hipGraphExec_t ge = nullptr;
  e = hipStreamEndCapture(st, &graph);
  if (e == hipSuccess) e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    *err = std::string("graph instantiate: ") + hipGetErrorString(e);
    if (graph) hipGraphDestroy(graph);
    return WBPR_EDEVICE;
  }
  graphs_[key] = {graph, ge};
  *exec = ge;
  return 0;
}

void Engine::dump_sweep_log(hipStream_t st) {
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  int32_t n = 0;
  if (hipMemcpyAsync(&n, &misc->log_n, 4, hipMemcpyDeviceToHost, st) != hipSuccess) return;
  if (hipStreamSynchronize(st) != hipSuccess) return;
  n = std::min(n, kSweepLogCap / 2);
  std::vector<int32_t> rec(6 * (size_t)std::max(n, 1));
  if (n > 0 && hipMemcpy(rec.data(), sweep_log_dev_, 24 * (size_t)n, hipMemcpyDeviceToHost) != hipSuccess) return;
  std::fprintf(stderr, "[wbpr] sweep log: %d sweeps (queue, medium, long, chunk tasks, queue out, relabel work)\n", n);
  for (int i = 0; i < n; i++)
    std::fprintf(stderr, "[wbpr] sweep %5d: %9d %8d %7d %8d %9d %11d\n", i, rec[6 * i], rec[6 * i + 1], rec[6 * i + 2],
                 rec[6 * i + 3], rec[6 * i + 4], rec[6 * i + 5]);
  hipMemsetAsync(&misc->log_n, 0, 4, st);
}

bool Engine::ensure_side() {
  if (side_) return true;
  if (external_) return false;  // creates nothing: the long-row chain stays on the solve stream
  hipStream_t s = nullptr;
  if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
  std::vector<hipEvent_t> ev(2 * 64, nullptr);
  for (auto &e : ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto &x : ev)
        if (x) hipEventDestroy(x);
      hipStreamDestroy(s);
      return false;
    }
  }
  side_ = s;
  fork_ev_ = std::move(ev);
  return true;
}

// tiers: bit 0 launches the medium-row kernel, bit 1 the long-row chunk
// kernels (the tile kernel and the control kernel always run).  With both,
// the long-row chain runs on the side stream beside the medium-row kernel:
// every queued vertex is in exactly one of the two lists, and the two touch
// shared state only through atomics, as workgroups of one kernel do.
void Engine::enqueue_sweeps(hipStream_t st, int K, int tiers) {
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  const bool rc = cfg_.rcsr;
  Graph g{(int32_t)Vcap_, HCAP, A_.rowb, A_.ent, A_.rev, rc ? A_.rev : nullptr, e_, h_, sink_, gap_hist_, misc->gap};
  // tile kernels: 512 workgroups, two per CU.  Measured on R-MAT / grid cut
  // / bipartite (means of three interleaved runs of nine solves): 256 ->
  // 26.0 / 70.9 / 4.55 ms, 512 -> 25.4 / 68.0 / 4.56, 1024 -> 26.1 / 72.0 /
  // 4.65; most sweeps have short queues, and each workgroup pays for its
  // start, its queue flushes and its counter atomics, while the big sweeps
  // after a global relabel want more waves in flight.  The long-row chunk
  // kernels keep 1024 (one workgroup per chunk task; 512 and 2048 measured
  // slower).
  const int sweep_blocks = cfg_.grid_blocks > 0 ? cfg_.grid_blocks : 512;
  static const int mid_env = std::getenv("WBPR_MID_BLOCKS") ? std::atoi(std::getenv("WBPR_MID_BLOCKS")) : 0;
  static const int chunk_env = std::getenv("WBPR_CHUNK_BLOCKS") ? std::atoi(std::getenv("WBPR_CHUNK_BLOCKS")) : 0;
  const int mid_blocks = mid_env > 0 ? mid_env : sweep_blocks;
  const int chunk_blocks = chunk_env > 0 ? chunk_env : 1024;
  const int mode = cfg_.push_mode == 1 ? 0 : 1;
  const bool timed = cfg_.time_kernels;
  const bool fs = cfg_.full_scan;
  const bool fork = !timed && (tiers & 3) == 3 && side_ != nullptr;
  for (int j = 0; j < K; j++) {
    SweepQ q{};
    q.qin = fs ? q_[1] : q_[j & 1];
    q.qin_cnt = fs ? &misc->scan_cnt : &misc->qcnt[j % 3];
    q.qout = fs ? q_[0] : q_[(j + 1) & 1];
    q.qout_cnt = fs ? &misc->qcnt[0] : &misc->qcnt[(j + 1) % 3];
    q.zero_cnt = fs ? &misc->qcnt[0] : &misc->qcnt[(j + 2) % 3];
    q.append = fs ? 0 : 1;
    q.mid_v = mid_;
    q.mid_cnt = &misc->mid_cnt[j & 1];
    q.big_v = big_;
    q.big_cnt = &misc->big_cnt[j & 1];
    q.task_u = task_u_;
    q.task_c = task_c_;
    q.task_cnt = &misc->task_cnt[j & 1];
    q.zero_c = &misc->task_cnt[(j + 1) & 1];
    q.tcap = (int32_t)std::min<int64_t>(tcap_, 0x7fffffff);
    q.lr_key = lr_key_;
    q.lr_cnt = lr_cnt_;
    q.zero_a = &misc->mid_cnt[(j + 1) & 1];
    q.zero_b = &misc->big_cnt[(j + 1) & 1];
    q.t_mid = t_mid_;
    q.t_big = t_big_;
    q.mode = mode;
    q.stats = misc->stats;
    q.gap_skips = &misc->stats[15];
    q.rwork = &misc->rwork;
    q.part = misc->part;
    q.sofs = 0;
    q.halt = &misc->halt[0];
    q.qcap = (int32_t)Vcap_;
    q.err = misc->err;
    q.wtrace = cfg_.wave_trace ? wtrace_ : nullptr;
    q.wtrace_n = &misc->wtrace_n;
    q.wtrace_cap = kTraceCap;
    q.sweep_no = &misc->sweep_no;
    q.kind = 0;
    SweepQ qw = q;
    qw.kind = 1;
    qw.qin = mid_;
    qw.qin_cnt = &misc->mid_cnt[j & 1];
    qw.zero_cnt = nullptr;
    qw.t_mid = 0x7fffffff;
    qw.t_big = 0x7fffffff;
    qw.sofs = 4;
    int evb = -1;
    if (timed) {
      if (ev_used_ + 4 > (int)ev_.size()) {
        const size_t old = ev_.size();
        ev_.resize(old + 1024);
        for (size_t i = old; i < ev_.size(); i++) hipEventCreate(&ev_[i]);
      }
      evb = ev_used_;
      ev_used_ += 4;
      ev_marks_.push_back({tiers << 4, evb});  // a sweep; which tiers ran
      hipEventRecord(ev_[evb], st);
    }
    if (fs)
      launch_avq_scan(sweep_blocks, st, g, &misc->span, q_[1], &misc->scan_cnt, (int32_t)Vcap_, misc->err,
                      &misc->halt[0]);
    launch_sweep_tile(P_, rc, sweep_blocks, st, g, q);
    if (fork) {
      hipEvent_t ef = fork_ev_[(2 * j) % fork_ev_.size()], ej = fork_ev_[(2 * j + 1) % fork_ev_.size()];
      hipEventRecord(ef, st);
      hipStreamWaitEvent(side_, ef, 0);
      launch_sweep_chunk(0, rc, chunk_blocks, side_, g, q);
      launch_sweep_chunk(1, rc, chunk_blocks, side_, g, q);
      launch_sweep_chunk(2, rc, 64, side_, g, q);
      hipEventRecord(ej, side_);
      launch_sweep_tile(mid_lanes_, rc, mid_blocks, st, g, qw);
      hipStreamWaitEvent(st, ej, 0);
    } else {
      if (timed) hipEventRecord(ev_[evb + 1], st);
      if (tiers & 1) launch_sweep_tile(mid_lanes_, rc, mid_blocks, st, g, qw);
      if (timed) hipEventRecord(ev_[evb + 2], st);
      if (tiers & 2) {
        launch_sweep_chunk(0, rc, chunk_blocks, st, g, q);
        launch_sweep_chunk(1, rc, chunk_blocks, st, g, q);
        launch_sweep_chunk(2, rc, 64, st, g, q);
      }
      if (timed) hipEventRecord(ev_[evb + 3], st);
    }
    SweepCtl ctl{};
    ctl.qin_cnt = q.qin_cnt;
    ctl.mid_cnt = q.mid_cnt;
    ctl.big_cnt = q.big_cnt;
    ctl.task_cnt = q.task_cnt;
    ctl.qout_cnt = q.qout_cnt;
    ctl.rwork = &misc->rwork;
    ctl.rwork_at_gr = &misc->rwork_at_gr;
    ctl.budget = budget_;
    ctl.halt = &misc->halt[0];
    ctl.scan_cnt = fs ? &misc->scan_cnt : nullptr;
    ctl.stag = misc->stag;
    ctl.stag_window = cfg_.gr_every_sweeps > 0 ? 0x7fffffff : stag_window_;
    ctl.log = sweep_log_;
    ctl.log_n = &misc->log_n;
    ctl.log_cap = kSweepLogCap / 2;
    ctl.sweep_no = q.wtrace ? &misc->sweep_no : nullptr;
    ctl.part = misc->part;
    ctl.stats = misc->stats;
    ctl.rwork_acc = &misc->rwork;
    launch_sweep_control(st, ctl);
  }
}

int Engine::round(hipStream_t st, std::vector<Finished> *done, std::string *err) {
  if (resident_ == 0) return 0;
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  // tiers from the resident graphs' mean row length (measured: 4 lanes for
  // the grid cut, 16 for R-MAT)
  const double mean_row = resident_V_ > 0 ? (double)resident_M_ / (double)resident_V_ : 1.0;
  int32_t longest = 0;  // longest row a sweep can meet
  for (int i = 0; i < ncap_; i++)
    if (inst_[i].used && inst_[i].phase < 3) longest = std::max(longest, inst_[i].maxdeg);
  // one lane per row when no row is longer than 16 (measured on the grid
  // cut: 96 vs 109 ms with tiles of 4), else tiles by the mean row length
  const int P = cfg_.lanes_per_vertex > 0 ? cfg_.lanes_per_vertex
                : longest <= 16           ? 1
                : mean_row <= 10.0        ? 4
                : mean_row <= 20.0        ? 8
                                          : 16;
  // lanes_per_vertex = 1 with no tier thresholds given is the paper's
  // thread-centric baseline (no medium or long tiers); otherwise one lane is
  // a short-row tier (rows up to split_degree, default 16)
  const bool tc = cfg_.lanes_per_vertex == 1 && cfg_.split_degree == 0 && cfg_.block_degree == 0;
  const int tm = tc ? 0x7fffffff : cfg_.split_degree > 0 ? cfg_.split_degree : (P == 1 ? 16 : 4 * P);
  const int tb = tc ? 0x7fffffff : std::max(tm, cfg_.block_degree > 0 ? cfg_.block_degree : 2048);
  // stagnation window (measured: R-MAT best at 4, where excess that will be
  // stranded keeps circulating among hubs; the grid cut at 32, where the
  // queue shrinks slowly and relabels are long BFSs; bipartite at 8)
  const int sw = cfg_.gr_stagnation > 0 ? cfg_.gr_stagnation : (mean_row <= 10.0 ? 32 : mean_row <= 20.0 ? 8 : 4);
  if (P != P_ || tm != t_mid_ || tb != t_big_ || sw != stag_window_) {
    P_ = P;
    t_mid_ = tm;
    t_big_ = tb;
    stag_window_ = sw;
    bfs_split_ = 8 * P;
    drop_graphs();
  }
  acc_.lanes = P_;
  acc_.split_degree = t_mid_;
  acc_.block_degree = t_big_;
  // roots / excluded terminals of every resident instance for its phase
  int32_t *hroots = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                                4 * (size_t)ncap_);
  int32_t *hrh = hroots + ncap_;
  int32_t *hex = hrh + ncap_;
  int nr = 0, sink = -1;
  for (int i = 0; i < ncap_; i++) {
    const Inst &I = inst_[i];
    if (!I.used || I.phase >= 3) continue;
    hroots[nr] = I.phase == 1 ? I.t : I.s;
    hrh[nr] = HCAP - I.V;
    hex[nr] = I.phase == 1 ? I.s : I.t;
    nr++;
  }
  if (nr == 1) sink = hroots[0];
  const double beta = cfg_.gr_work_permille > 0 ? cfg_.gr_work_permille / 1000.0 : gr_beta_env();
  long long *hmisc = reinterpret_cast<long long *>(pin_ + 512);
  // the relabel and the full-scan queue visit vertices up to the end of the
  // highest resident group (free vertices below it are inactive, empty rows)
  int64_t vhi = 0;
  for (const Group &G : groups_)
    if (G.used) vhi = std::max<int64_t>(vhi, (int64_t)G.vbase + G.V);
  if (cfg_.debug_checks) {
    const int rc = debug_check(st, (int32_t)vhi, err);
    if (rc) return rc;
  }
  hmisc[0] = sink;
  hmisc[2] = vhi;
  hmisc[1] = cfg_.gr_every_sweeps > 0 ? (1LL << 62) : (long long)(beta * (double)(resident_V_ + resident_M_));
  // the same arguments as the last round's (one instance: every round of a
  // phase) are already on the device: each copy costs a blit on the stream
  std::vector<int64_t> up;
  up.reserve(3 * (size_t)nr + 4);
  up.push_back(nr);
  for (int i = 0; i < nr; i++) {
    up.push_back(hroots[i]);
    up.push_back(hrh[i]);
    up.push_back(hex[i]);
  }
  up.push_back(hmisc[0]);
  up.push_back(hmisc[1]);
  up.push_back(hmisc[2]);
  if (up != gr_uploaded_) {
    hipMemcpyAsync(roots_, hroots, 4 * (size_t)nr, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(root_h_, hrh, 4 * (size_t)nr, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(excl_, hex, 4 * (size_t)nr, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(sink_, &hmisc[0], 4, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(budget_, &hmisc[1], 8, hipMemcpyHostToDevice, st);
    hipMemcpyAsync(&misc->span, &hmisc[2], 4, hipMemcpyHostToDevice, st);
    gr_uploaded_ = std::move(up);
  }
  // status and the per-instance counts are cleared by the relabel itself

  Graph g{(int32_t)vhi, HCAP, A_.rowb, A_.ent, A_.rev, cfg_.rcsr ? A_.rev : nullptr, e_, h_, sink_, gap_hist_,
          misc->gap};
  GRArgs ga{};
  ga.g = g;
  ga.roots = roots_;
  ga.root_h = root_h_;
  ga.nroots = nr;
  ga.excl = excl_;
  ga.nexcl = nr;
  ga.inst_of = inst_of_;
  ga.inst_active = inst_active_;
  ga.ninst = ncap_;
  ga.inst_stranded = inst_stranded_;
  ga.fq[0] = fq_[0];
  ga.fq[1] = fq_[1];
  ga.fcnt = misc->fcnt;
  ga.vis = vis_;
  ga.chunk_w = chunk_w_;
  ga.chunk_b = chunk_b_;
  ga.chunk_cnt = misc->chunk_cnt;
  ga.bucnt = misc->bucnt;
  ga.fedges = misc->fedges;
  ga.bar = misc->bar;
  ga.qout = q_[0];
  ga.qcnt = misc->qcnt;
  ga.big_cnt = misc->big_cnt;
  ga.mid_cnt = misc->mid_cnt;
  ga.task_cnt = misc->task_cnt;
  ga.stats = misc->stats;
  ga.status = misc->status;
  ga.split_deg = bfs_split_;
  ga.chunk = chunk_;
  ga.qcap = (int32_t)Vcap_;
  ga.chunk_cap = (int32_t)std::min<int64_t>(nchunk_, 0x7fffffff);
  ga.bu_threshold = (int32_t)std::max<int64_t>(resident_V_ / 32, 4096);
  ga.bu_edges = std::max<long long>(resident_M_ / 16, 65536);
  ga.m_total = resident_M_;
  ga.err = misc->err;
  ga.halt = misc->halt;
  ga.rwork = &misc->rwork;
  ga.rwork_at_gr = &misc->rwork_at_gr;
  ga.stag = misc->stag;
  // the medium-row list is idle during a relabel: it holds the bitmaps
  // (4 x ceil(V/32) words <= V words)
  ga.bm = reinterpret_cast<uint32_t *>(mid_);
  ga.bm_words = (int32_t)((Vcap_ + 31) / 32);
  // diagnostics (WBPR_LOG >= 3): per-level timestamps in the sweep-log space
  // second half of the sweep-log space (the sweep log keeps the first)
  ga.tlog = log_level() >= 3 ? reinterpret_cast<long long *>(sweep_log_dev_ + 3 * (size_t)kSweepLogCap) : nullptr;
  ga.tlog_cap = kSweepLogCap / 2;
  // gap heuristic: exact per-height counts need one root (one instance in
  // its phase); batches run without it
  ga.gap_base = nr == 1 ? hrh[0] : 0;
  ga.gap_n = cfg_.gap && nr == 1 ? std::min(HCAP - hrh[0], GAP_BINS) : 0;
  const int Pg = std::max(P_, 4);  // tile width of the relabel's top-down expansion
  int lg = 0;
  while ((1 << lg) < Pg) lg++;
  const int gr_blocks = std::min(gr_blocks_[lg], 1024);
  acc_.gr_blocks = gr_blocks;
  if (gr_blocks < 1) {
    *err = "cooperative launch not possible";
    return WBPR_EDEVICE;
  }
  auto tg0 = std::chrono::steady_clock::now();
  int evb = -1;
  if (cfg_.time_kernels) {
    if (ev_used_ + 2 > (int)ev_.size()) {
      const size_t old = ev_.size();
      ev_.resize(old + 1024);
      for (size_t i = old; i < ev_.size(); i++) hipEventCreate(&ev_[i]);
    }
    evb = ev_used_;
    ev_used_ += 2;
    ev_marks_.push_back({3, evb});
    hipEventRecord(ev_[evb], st);
  }
  hipError_t he = launch_global_relabel(Pg, cfg_.rcsr, gr_blocks, st, ga);
  if (he != hipSuccess) {
    *err = std::string("global relabel launch: ") + hipGetErrorString(he);
    return WBPR_EDEVICE;
  }
  if (evb >= 0) hipEventRecord(ev_[evb + 1], st);
  acc_.global_relabels++;
  // read back: status (4 x i64), err (2 x i32), per-instance counts
  char *rb = pin_ + 2048;
  he = hipMemcpyAsync(rb, misc->status, sizeof(misc->status) + sizeof(misc->err), hipMemcpyDeviceToHost, st);
  int32_t *hact = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                              16 * (size_t)ncap_);
  int32_t *hstr = hact + ncap_;
  if (he == hipSuccess) he = hipMemcpyAsync(hact, inst_active_, 4 * (size_t)ncap_, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(hstr, inst_stranded_, 4 * (size_t)ncap_, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipMemcpyAsync(rb + 64, &misc->stats[13], 8, hipMemcpyDeviceToHost, st);
  if (he == hipSuccess) he = hipStreamSynchronize(st);
  if (he != hipSuccess) {
    *err = std::string("global relabel: ") + hipGetErrorString(he);
    return WBPR_EDEVICE;
  }
  const long long *status = reinterpret_cast<const long long *>(rb);
  const int32_t *errw = reinterpret_cast<const int32_t *>(rb + sizeof(misc->status));
  if (ga.tlog) {  // per-level times of this relabel (100 MHz wall clock)
    const int nl = (int)std::min<long long>(status[2] + 3, ga.tlog_cap);
    std::vector<long long> t(3 * (size_t)nl);
    if (hipMemcpy(t.data(), ga.tlog, 24 * (size_t)nl, hipMemcpyDeviceToHost) == hipSuccess) {
      std::string line = "[wbpr] relabel levels (us, frontier, frontier edges; negative: bottom-up):";
      for (int i = 1; i < nl; i++) {
        char buf[96];
        std::snprintf(buf, sizeof(buf), " [%.1f %lld %lld]", (t[3 * i] - t[3 * (i - 1)]) / 100.0, t[3 * (i - 1) + 1],
                      t[3 * (i - 1) + 2]);
        line += buf;
      }
      std::fprintf(stderr, "%s\n", line.c_str());
    }
  }
  acc_.gr_levels += status[2];
  if (log_level() > 0) {
    const double gms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - tg0).count();
    std::fprintf(stderr,
                 "[wbpr] round %lld: roots=%d active=%lld stranded=%lld bfs_levels=%lld (bottom-up %lld) "
                 "sweeps+gr+sync=%.3f ms\n",
                 (long long)acc_.global_relabels, nr, status[0], status[1], status[2], status[3], gms);
  }
  if (errw[0] != 0) {
    *err = "internal queue overflow";
    return WBPR_EINTERNAL;
  }
  // per-instance transitions
  std::vector<int> fin1, fin2, to2, fin_done;
  for (int i = 0; i < ncap_; i++) {
    Inst &I = inst_[i];
    if (!I.used || I.phase >= 3) continue;
    if (I.phase == 2 && hstr[i] > 0) {
      *err = "second phase: excess that cannot return to the source";
      return WBPR_EINTERNAL;
    }
    if (hact[i] != 0) continue;
    if (I.phase == 1) {
      fin1.push_back(i);
      if (I.flow) to2.push_back(i);
      else fin_done.push_back(i);
    } else {
      fin2.push_back(i);
      fin_done.push_back(i);
    }
  }
  launch_inst_kernel(IK_VALUE_ZERO, fin1, st);
  launch_inst_kernel(IK_VALUE, fin1, st);
  launch_inst_kernel(IK_SIDE, fin1, st);
  launch_inst_kernel(IK_PHASE2, to2, st);
  launch_inst_kernel(IK_DECODE, fin2, st);
  for (int i : to2) inst_[i].phase = 2;
  for (int i : fin_done) inst_[i].phase = 3;
  // sweeps for the instances still active.  A round starts with a batch
  // sized to the sweeps that found work in the last round (an empty sweep
  // slot after the device halts still costs its launches); while a batch
  // runs to its end without a halt the round goes on with one twice as long,
  // up to 72 sweeps in the round (heights older than that cost more sweeps
  // than a relabel on the grid cut), so no relabel is spent on a batch that
  // was merely short.
  // The device ends a batch early on an empty queue, the relabel budget or
  // stagnation.  Batch lengths are multiples of 6: sweep j takes its queue
  // count from slot j % 3 and its lists from slot j % 2, so such a batch
  // leaves the rings where the next batch's first sweep starts.
  long long nonempty = 0;
  std::memcpy(&nonempty, rb + 64, 8);
  const long long ran = nonempty - last_nonempty_;
  last_nonempty_ = nonempty;
  if (last_K_ > 0) {
    int k = 6;
    while (k < ran) k *= 2;
    next_K_ = std::min(k, 48);
  }
  if (status[0] > 0) {
    const bool fixed = cfg_.gr_every_sweeps > 0;
    int K = fixed ? cfg_.gr_every_sweeps : next_K_;
    last_K_ = K;
    // tiers that no resident row can reach are not launched
    int32_t rows = 0;
    for (int i = 0; i < ncap_; i++)
      if (inst_[i].used && inst_[i].phase < 3) rows = std::max(rows, inst_[i].maxdeg);
    const int tiers = (rows > t_mid_ ? 1 : 0) | (rows > t_big_ ? 2 : 0);
    if ((tiers & 3) == 3) ensure_side();  // before any capture begins
    if (cfg_.wave_trace && !wtrace_ && hipMalloc(&wtrace_, 16 * (size_t)kTraceCap) != hipSuccess) {
      wtrace_ = nullptr;
      *err = "out of device memory for the wave trace";
      return WBPR_ENOMEM;
    }
    int32_t *hhalt = reinterpret_cast<int32_t *>(rb + 96);
    for (int total = 0;;) {
      if (cfg_.use_graph && !cfg_.time_kernels) {
        hipGraphExec_t exec = nullptr;
        int rc = ensure_graph(st, K, tiers, &exec, err);
        if (rc) return rc;
        he = hipGraphLaunch(exec, st);
        if (he != hipSuccess) {
          *err = std::string("graph launch: ") + hipGetErrorString(he);
          return WBPR_EDEVICE;
        }
      } else {
        enqueue_sweeps(st, K, tiers);
      }
      acc_.sweeps += K;
      total += K;
      const int more = std::min(2 * K, 72 - total) / 6 * 6;
      if (fixed || more <= 0) break;
      he = hipMemcpyAsync(hhalt, &misc->halt[0], 4, hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) {
        *err = std::string("sweeps: ") + hipGetErrorString(he);
        return WBPR_EDEVICE;
      }
      if (*hhalt) break;
      K = more;
    }
  }
  he = hipGetLastError();
  if (he != hipSuccess) {
    *err = std::string("launch: ") + hipGetErrorString(he);
    return WBPR_EDEVICE;
  }
  // instances solved whole at admission retire with this round's
  for (int i = 0; i < ncap_; i++)
    if (inst_[i].used && inst_[i].pending_done) {
      inst_[i].pending_done = false;
      fin_done.push_back(i);
    }
  retire(fin_done, done, st);
  return 0;
}

// Hands out finished instances, frees their slots and releases groups that
// have no instance left (parks kept ones).
void Engine::retire(const std::vector<int> &fin_done, std::vector<Finished> *done, hipStream_t st) {
  std::vector<int> empty_groups;
  std::vector<InstDev> parked;
  for (int i : fin_done) {
    Inst &I = inst_[i];
    Group &G = groups_[I.group];
    done->push_back(Finished{G.tag, I.index, 0});
    G.remaining--;
    if (G.remaining == 0 && !G.keep) empty_groups.push_back(I.group);
    if (G.remaining == 0 && G.keep) {
      InstDev d;
      std::memset(&d, 0, sizeof(d));
      d.vbase = G.vbase;
      d.V = G.V;
      parked.push_back(d);
    }
    I = Inst();
    slot_free_.push_back(i);
    resident_--;
  }
  release_groups(empty_groups, st);
  if (!parked.empty()) launch_inst_list(IK_PARK, parked, std::vector<int>(parked.size(), 0), st);
}

// ------------------------------------------------- persistent kernel, live

constexpr double kPkIdleMs = 2.0;  // a workgroup exits after this long without an entry

int Engine::pk_publish(const std::vector<int> &slots, hipStream_t st, std::string *err) {
  std::vector<int> cand;
  for (int sl : slots) {
    Inst &I = inst_[sl];
    if (I.phase == 1 && I.V <= WG_MAX_V && I.E <= WG_MAX_E) cand.push_back(sl);
  }
  if (cand.empty()) return 0;
  std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return inst_[a].E > inst_[b].E; });
  const int n = (int)cand.size();
  if ((int64_t)pk_out_.size() + n > ncap_) {  // cannot happen: a ring slot per resident instance
    *err = "persistent ring overflow";
    return WBPR_EINTERNAL;
  }
  WgInst *hl = reinterpret_cast<WgInst *>(reinterpret_cast<InstDev *>(pin_ + kPinnedHeader) + (size_t)IK_WG * ncap_);
  for (int i = 0; i < n; i++) fill_wg(inst_[cand[i]], &hl[i]);
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  hipError_t e = hipMemcpyAsync(pk_stage_, hl, sizeof(WgInst) * n, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    launch_pk_publish(st, pk_stage_, n, pk_ring_, ncap_, pk_result_, &misc->pk_tail);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the pinned slice is reused by the next publish
  if (e != hipSuccess) {
    *err = std::string("persistent publish: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  for (int i = 0; i < n; i++) {
    inst_[cand[i]].phase = 4;
    pk_out_.push_back({pk_tail_ + i, cand[i]});
  }
  pk_tail_ += n;
  return 0;
}

bool Engine::pk_alive() {
  if (!pk_launched_) return false;
  if (hipEventQuery(pk_ev_) == hipSuccess) pk_launched_ = false;
  return pk_launched_;
}

int Engine::pk_ensure_running(hipStream_t st_pk, std::string *err) {
  if (pk_out_.empty() || pk_alive()) return 0;
  if (!pk_ev_ && hipEventCreateWithFlags(&pk_ev_, hipEventDisableTiming) != hipSuccess) {
    pk_ev_ = nullptr;
    *err = "persistent kernel event";
    return WBPR_EDEVICE;
  }
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  WgArgs a{};
  a.L = pk_ring_;
  a.n = 0;
  a.head = &misc->pk_head;
  a.tail = &misc->pk_tail;
  a.close = nullptr;
  a.idle_ticks = (long long)(kPkIdleMs * 1e5);  // 100 MHz device clock
  a.ring = ncap_;
  a.result = pk_result_;
  a.rowb = A_.rowb;
  a.ent = A_.ent;
  a.rev = A_.rev;
  a.cap0 = A_.cap0;
  a.arc2ent = A_.arc2ent;
  a.pbefore = A_.pbefore;
  a.acap = A_.acap;
  a.e = e_;
  a.h = h_;
  a.qa = q_[0];
  a.qb = q_[1];
  a.stats = misc->wg_stats;
  a.round_cap = 0;
  a.max_ticks = (long long)(kWgMaxMs * 1e5);
  // two workgroups per CU: the other wave slots stay free for the
  // admissions' builder kernels on the server stream
  int ncu = 256;
  hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device_);
  launch_wg_solve(cfg_.rcsr, 2 * ncu, st_pk, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(pk_ev_, st_pk);
  if (e != hipSuccess) {
    *err = std::string("persistent kernel launch: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  pk_launched_ = true;
  return 0;
}

int Engine::pk_collect(hipStream_t st, std::vector<Finished> *done, std::string *err) {
  if (pk_out_.empty()) return 0;
  int32_t *hres = reinterpret_cast<int32_t *>(pin_ + kPinnedHeader + sizeof(InstDev) * (size_t)ncap_ * kListKinds +
                                              8 * (size_t)ncap_);
  hipError_t e = hipMemcpyAsync(hres, pk_result_, 4 * (size_t)ncap_, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = std::string("persistent results: ") + hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  std::vector<int> fin;
  std::vector<std::pair<int32_t, int>> keep;
  for (const auto &it : pk_out_) {
    const int32_t r = hres[it.first % ncap_];
    Inst &I = inst_[it.second];
    if (r == 1) {
      I.phase = 3;
      fin.push_back(it.second);
      acc_.wg_solved++;
    } else if (r == 2 || r == 3) {  // stopped at a cap: the rounds finish it
      I.phase = r == 3 ? 2 : 1;
      acc_.wg_fallbacks++;
    } else {
      keep.push_back(it);
    }
  }
  pk_out_.swap(keep);
  retire(fin, done, st);
  return 0;
}

int32_t Engine::rounds_resident() const {
  int32_t n = 0;
  for (const Inst &I : inst_)
    if (I.used && (I.phase == 1 || I.phase == 2)) n++;
  return n;
}


int Engine::run_to_completion(hipStream_t st, std::vector<Finished> *done, std::string *err) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t sweeps0 = acc_.sweeps;
  while (resident_ > 0) {
    int rc = round(st, done, err);
    if (rc) return rc;
    if (cfg_.max_sweeps > 0 && acc_.sweeps - sweeps0 > cfg_.max_sweeps) {
      *err = "max_sweeps exceeded";
      return WBPR_ETIMEOUT;
    }
    if (cfg_.max_wall_ms > 0 &&
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > cfg_.max_wall_ms) {
      *err = "max_wall_ms exceeded";
      return WBPR_ETIMEOUT;
    }
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  if (sweep_log_) dump_sweep_log(st);
  return 0;
}

void Engine::abandon(hipStream_t st) {
  hipStreamSynchronize(st);
  if (misc_ && !pk_out_.empty()) {
    // the persistent kernel has exited (callers wait for it): entries still
    // in its ring are skipped, so a later launch never claims them
    MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
    hipMemcpyAsync(&misc->pk_head, &misc->pk_tail, sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  }
  pk_out_.clear();
  if (arena_) {
    hipMemsetAsync(A_.rowb, 0, 8 * (size_t)Vcap_, st);
    hipMemsetAsync(e_, 0, 8 * (size_t)Vcap_, st);
    hipMemsetAsync(inst_of_, 0xff, 4 * (size_t)Vcap_, st);
    hipStreamSynchronize(st);
  }
  valloc_.reset(Vcap_);
  malloc_.reset(Mcap_);
  aalloc_.reset(Ecap_);
  slot_free_.clear();
  for (int32_t i = ncap_ - 1; i >= 0; i--) slot_free_.push_back(i);
  inst_.assign(ncap_, Inst());
  groups_.clear();
  resident_ = 0;
  resident_V_ = 0;
  resident_M_ = 0;
}

void Engine::reset_stats() {
  acc_ = EngineStats();
  next_K_ = 12;
  last_K_ = 0;
  ev_used_ = 0;
  ev_marks_.clear();
  last_nonempty_ = 0;
  if (misc_) {
    MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
    hipMemset(misc->stats, 0, sizeof(misc->stats));
    hipMemset(misc->part, 0, sizeof(misc->part));
    hipMemset(&misc->wtrace_n, 0, 2 * sizeof(int32_t));
    hipMemset(misc->wg_stats, 0, sizeof(misc->wg_stats));
  }
}

int64_t Engine::read_wave_trace(hipStream_t st, int32_t *host, int64_t cap, std::string *err) {
  if (!wtrace_ || !misc_) return 0;
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  int32_t n = 0;
  hipError_t e = hipMemcpyAsync(pin_ + 3072, &misc->wtrace_n, 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return -1;
  }
  std::memcpy(&n, pin_ + 3072, 4);
  const int64_t kept = std::min<int64_t>(n, kTraceCap);
  const int64_t k = std::min<int64_t>(kept, cap);
  if (k > 0) {
    e = hipMemcpyAsync(host, wtrace_, 16 * (size_t)k, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      *err = hipGetErrorString(e);
      return -1;
    }
  }
  return kept;
}

int Engine::collect_stats(hipStream_t st, EngineStats *out, std::string *err) {
  MiscLayout *misc = reinterpret_cast<MiscLayout *>(misc_);
  long long hs[16];
  hipError_t e = hipMemcpyAsync(pin_ + 3072, misc->stats, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  std::memcpy(hs, pin_ + 3072, sizeof(hs));
  EngineStats r = acc_;
  for (int k = 0; k < 3; k++) {
    r.k_scans[k] = hs[4 * k + 0];
    r.k_pushes[k] = hs[4 * k + 1];
    r.k_relabels[k] = hs[4 * k + 2];
    r.k_queued[k] = hs[4 * k + 3];
    r.arc_scans += r.k_scans[k];
    r.pushes += r.k_pushes[k];
    r.relabels += r.k_relabels[k];
    r.queued += r.k_queued[k];
  }
  r.k_scans[3] = hs[12] + hs[14];
  r.bfs_scans = hs[12] + hs[14];
  r.bfs_topdown_scans = hs[12];
  r.nonempty_sweeps = hs[13];
  r.gap_skipped = hs[15];
  long long wg[6];
  e = hipMemcpy(wg, misc->wg_stats, sizeof(wg), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    *err = hipGetErrorString(e);
    return WBPR_EDEVICE;
  }
  // the persistent kernel's sweeps count with the short-row tile kernel's,
  // its BFS rounds with the global relabels
  r.k_scans[0] += wg[0];
  r.k_pushes[0] += wg[1];
  r.k_relabels[0] += wg[2];
  r.arc_scans += wg[0];
  r.pushes += wg[1];
  r.relabels += wg[2];
  r.sweeps += wg[3];
  r.global_relabels += wg[4];
  r.bfs_scans += wg[5];
  for (const auto &mk : ev_marks_) {
    if (mk.first == 5) {  // residual-graph build
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev_[mk.second], ev_[mk.second + 1]) == hipSuccess) r.build_ms += ms;
      continue;
    }
    if (mk.first == 3) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev_[mk.second], ev_[mk.second + 1]) == hipSuccess) r.k_ms[3] += ms;
      r.k_launches[3]++;
    } else {
      const int tiers = mk.first >> 4;
      for (int k = 0; k < 3; k++) {
        if (k == 1 && !(tiers & 1)) continue;  // tier not launched in this sweep
        if (k == 2 && !(tiers & 2)) continue;
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev_[mk.second + k], ev_[mk.second + k + 1]) == hipSuccess) r.k_ms[k] += ms;
        r.k_launches[k]++;
      }
    }
  }
  *out = r;
  return 0;
}

}  // namespace wb
