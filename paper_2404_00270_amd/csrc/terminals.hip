// Source/sink selection and multi-terminal solves: the experimental protocol
// of the paper (section 4).  Graphs without given terminals get source/sink
// pairs chosen by breadth-first search among those farthest apart, and a
// super-source and a super-sink joined to all of them turn the multi-source,
// multi-sink problem into one s-t maximum flow.
//
// The search is a bit-parallel BFS over the arcs of positive capacity: up
// to 64 sources share one pass, seen[v] holding bit b once source b has
// reached v and front[v] the bits that reached v at the current level.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <vector>

#include "wb_common.h"
#include "wb_ctx.h"

namespace wb {
namespace {

constexpr int TB = 256;

// Device buffer owned by one call: waits for the stream, then frees.
struct TmpBuf {
  DevBuf b;
  hipStream_t st;
  explicit TmpBuf(hipStream_t s) : st(s) {}
  ~TmpBuf() {
    if (b.p) {
      hipStreamSynchronize(st);
      b.release();
    }
  }
  TmpBuf(const TmpBuf &) = delete;
  TmpBuf &operator=(const TmpBuf &) = delete;
};

unsigned grid_of(int64_t n) {
  int64_t b = (n + TB - 1) / TB;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

__device__ __forceinline__ unsigned long long far_key(int32_t level, int32_t v) {
  // larger level first, then the smaller vertex id
  return ((unsigned long long)(uint32_t)level << 32) | (uint32_t)~(uint32_t)v;
}

__global__ void k_ms_init(const int32_t *src, int32_t nb, unsigned long long *seen, unsigned long long *front,
                          unsigned long long *far) {
  const int b = threadIdx.x;
  if (b < nb) {
    atomicOr(&seen[src[b]], 1ull << b);
    atomicOr(&front[src[b]], 1ull << b);
    far[b] = far_key(0, src[b]);
  }
}

// Level step 1: every vertex with new bits offers them to its out-neighbours
// along arcs of positive capacity.
__global__ void k_ms_expand(const int64_t *rp, const int32_t *col, const int32_t *cap, int32_t V,
                            const unsigned long long *front, const unsigned long long *seen,
                            unsigned long long *next) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long f = front[v];
    if (!f) continue;
    for (int64_t a = rp[v], end = rp[v + 1]; a < end; a++) {
      if (cap[a] <= 0) continue;
      const int32_t w = col[a];
      const unsigned long long nw = f & ~seen[w];
      if (nw) atomicOr(&next[w], nw);
    }
  }
}

// Level step 2: bits that reach a vertex for the first time form its new
// front; each source keeps the farthest vertex it has reached (largest
// level, then smallest id), and alive collects the sources still growing.
__global__ void k_ms_update(int32_t V, int32_t level, unsigned long long *front, unsigned long long *seen,
                            unsigned long long *next, unsigned long long *far, unsigned long long *alive) {
  unsigned long long any = 0;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < V; w += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long n = next[w] & ~seen[w];
    next[w] = 0;
    front[w] = n;
    if (n) {
      seen[w] |= n;
      any |= n;
      const unsigned long long key = far_key(level, (int32_t)w);
      for (unsigned long long m = n; m; m &= m - 1) atomicMax(&far[__ffsll((long long)m) - 1], key);
    }
  }
#pragma unroll
  for (int m = WB_WAVE / 2; m > 0; m >>= 1) any |= shfl_xor_u64(any, m);
  if (lane() == 0 && any) atomicOr(alive, any);
}

// Eccentricity (largest BFS distance over arcs of positive capacity) and the
// farthest vertex (smallest id among those at that distance) of every vertex
// in from[0..n), on a CSR already in device memory.
int bfs_farthest_dev(hipStream_t st, const int64_t *rp, const int32_t *col, const int32_t *cap, int32_t V, int32_t n,
                     const int32_t *from, int32_t *ecc, int32_t *farthest, int max_wall_ms) {
  const auto t0 = std::chrono::steady_clock::now();
  TmpBuf bits_(st), aux_(st);
  DevBuf &bits = bits_.b, &aux = aux_.b;
  hipError_t e = bits.ensure(24 * (size_t)V);
  if (e == hipSuccess) e = aux.ensure(8 * 64 + 8 + 4 * 64);
  if (e != hipSuccess) return hip_fail(e, "bfs buffers");
  unsigned long long *seen = (unsigned long long *)bits.p, *front = seen + V, *next = front + V;
  unsigned long long *far = (unsigned long long *)aux.p, *alive = far + 64;
  int32_t *src = (int32_t *)(alive + 1);
  std::vector<unsigned long long> hfar(64);
  for (int32_t b0 = 0; b0 < n; b0 += 64) {
    const int32_t nb = std::min<int32_t>(64, n - b0);
    e = hipMemsetAsync(bits.p, 0, 24 * (size_t)V, st);
    if (e == hipSuccess) e = hipMemcpyAsync(src, from + b0, 4 * (size_t)nb, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "bfs init");
    hipLaunchKernelGGL(k_ms_init, dim3(1), dim3(64), 0, st, src, nb, seen, front, far);
    for (int32_t level = 1;; level++) {
      unsigned long long halive = 0;
      e = hipMemsetAsync(alive, 0, 8, st);
      if (e != hipSuccess) return hip_fail(e, "bfs level");
      hipLaunchKernelGGL(k_ms_expand, dim3(grid_of(V)), dim3(TB), 0, st, rp, col, cap, V, front, seen, next);
      hipLaunchKernelGGL(k_ms_update, dim3(grid_of(V)), dim3(TB), 0, st, V, level, front, seen, next, far, alive);
      e = hipMemcpyAsync(&halive, alive, 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "bfs level");
      if (halive == 0) break;
      if (max_wall_ms > 0 &&
          std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() > max_wall_ms)
        return fail(WBPR_ETIMEOUT, "max_wall_ms exceeded");
    }
    e = hipMemcpyAsync(hfar.data(), far, 8 * (size_t)nb, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "bfs result");
    for (int32_t b = 0; b < nb; b++) {
      ecc[b0 + b] = (int32_t)(hfar[b] >> 32);
      farthest[b0 + b] = (int32_t)~(uint32_t)hfar[b];
    }
  }
  return WBPR_OK;
}

// Host CSR -> device copies (row pointers, columns, capacities).
struct DevCsr {
  TmpBuf rp_, col_, cap_;
  DevBuf &rp = rp_.b, &col = col_.b, &cap = cap_.b;
  explicit DevCsr(hipStream_t st) : rp_(st), col_(st), cap_(st) {}
  int upload(const wbpr_csr *g, hipStream_t st) {
    hipError_t e = rp.ensure(8 * ((size_t)g->V + 1));
    if (e == hipSuccess) e = col.ensure(4 * (size_t)std::max<int64_t>(g->E, 1));
    if (e == hipSuccess) e = cap.ensure(4 * (size_t)std::max<int64_t>(g->E, 1));
    if (e == hipSuccess) e = hipMemcpyAsync(rp.p, g->row_ptr, 8 * ((size_t)g->V + 1), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && g->E > 0) e = hipMemcpyAsync(col.p, g->col, 4 * (size_t)g->E, hipMemcpyHostToDevice, st);
    if (e == hipSuccess && g->E > 0) e = hipMemcpyAsync(cap.p, g->cap, 4 * (size_t)g->E, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(e, "graph upload");
    return WBPR_OK;
  }
};

// Host-side checks of a CSR for the BFS (the solver validates on the device).
int check_csr_host(const wbpr_csr *g) {
  if (!g || g->V <= 0 || g->E < 0 || !g->row_ptr || (g->E > 0 && (!g->col || !g->cap)))
    return fail(WBPR_EINVAL, "invalid graph");
  if (g->row_ptr[0] != 0 || g->row_ptr[g->V] != g->E) return fail(WBPR_EINVAL, "row pointers");
  for (int32_t v = 0; v < g->V; v++)
    if (g->row_ptr[v + 1] < g->row_ptr[v]) return fail(WBPR_EINVAL, "row pointers");
  for (int64_t a = 0; a < g->E; a++)
    if (g->col[a] < 0 || g->col[a] >= g->V) return fail(WBPR_EINVAL, "column out of range");
  return WBPR_OK;
}

// SplitMix64 (Steele, Lea and Flood, 2014): the candidate draws.
uint64_t splitmix64(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

}  // namespace
}  // namespace wb

using namespace wb;

extern "C" {

int wbpr_bfs_farthest(wbpr_ctx *c, const wbpr_csr *g, int32_t n, const int32_t *from, int32_t *ecc,
                      int32_t *farthest) {
  if (!c || !g || n < 0 || (n > 0 && (!from || !ecc || !farthest))) return fail(WBPR_EINVAL, "null argument");
  int rc = check_csr_host(g);
  if (rc) return rc;
  for (int32_t i = 0; i < n; i++)
    if (from[i] < 0 || from[i] >= g->V) return fail(WBPR_EINVAL, "source out of range");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  DevCsr d(c->stream);
  rc = d.upload(g, c->stream);
  if (rc) return rc;
  return bfs_farthest_dev(c->stream, (const int64_t *)d.rp.p, (const int32_t *)d.col.p, (const int32_t *)d.cap.p,
                          g->V, n, from, ecc, farthest, c->cfg.max_wall_ms);
}

int wbpr_pick_terminals(wbpr_ctx *c, const wbpr_csr *g, int32_t k, uint64_t seed, int32_t *sources,
                        int32_t *sinks, int32_t *npairs) {
  if (!c || !g || k < 0 || !npairs || (k > 0 && (!sources || !sinks))) return fail(WBPR_EINVAL, "null argument");
  int rc = check_csr_host(g);
  if (rc) return rc;
  *npairs = 0;
  // candidates: 4k distinct vertices with an arc of positive capacity,
  // drawn in SplitMix64 order (at most 64 draws per wanted candidate)
  std::vector<uint8_t> out_pos((size_t)g->V, 0);
  int64_t n_out = 0;
  for (int32_t v = 0; v < g->V; v++) {
    for (int64_t a = g->row_ptr[v]; a < g->row_ptr[v + 1]; a++)
      if (g->cap[a] > 0 && g->col[a] != v) {
        out_pos[v] = 1;
        break;
      }
    n_out += out_pos[v];
  }
  const int64_t want = std::min<int64_t>(4 * (int64_t)k, n_out);
  std::vector<int32_t> cand;
  std::vector<uint8_t> drawn((size_t)g->V, 0);
  uint64_t x = seed;
  for (int64_t tries = 0; (int64_t)cand.size() < want && tries < 64 * want; tries++) {
    const int32_t v = (int32_t)(splitmix64(&x) % (uint64_t)g->V);
    if (!out_pos[v] || drawn[v]) continue;
    drawn[v] = 1;
    cand.push_back(v);
  }
  if (cand.empty()) return WBPR_OK;
  std::vector<int32_t> ecc(cand.size()), far(cand.size());
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  DevCsr d(c->stream);
  rc = d.upload(g, c->stream);
  if (rc) return rc;
  rc = bfs_farthest_dev(c->stream, (const int64_t *)d.rp.p, (const int32_t *)d.col.p, (const int32_t *)d.cap.p, g->V,
                        (int32_t)cand.size(), cand.data(), ecc.data(), far.data(), c->cfg.max_wall_ms);
  if (rc) return rc;
  // longest eccentricities first (draw order on ties); pairs use distinct vertices
  std::vector<int32_t> order(cand.size());
  for (size_t i = 0; i < order.size(); i++) order[i] = (int32_t)i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ecc[a] > ecc[b]; });
  std::vector<uint8_t> used((size_t)g->V, 0);
  int32_t m = 0;
  for (int32_t i : order) {
    if (m == k || ecc[i] == 0) break;
    const int32_t s = cand[i], t = far[i];
    if (used[s] || used[t]) continue;
    used[s] = used[t] = 1;
    sources[m] = s;
    sinks[m] = t;
    m++;
  }
  *npairs = m;
  return WBPR_OK;
}

int wbpr_solve_multi(wbpr_ctx *c, const wbpr_csr *g, int32_t k, const int32_t *sources, const int32_t *sinks,
                     int64_t *value, int32_t *arc_flow, uint8_t *cut_side, wbpr_stats *stats) {
  if (!c || !g || !value || k <= 0 || !sources || !sinks) return fail(WBPR_EINVAL, "null argument");
  int rc = check_csr_host(g);
  if (rc) return rc;
  const int32_t V = g->V;
  const int64_t E = g->E;
  if ((int64_t)V + 2 >= (1ll << 31) - 1 || E + 2 * (int64_t)k >= (1ll << 31) - 1) return fail(WBPR_ETOOBIG, "too big");
  // role of every vertex: 1 source, 2 sink; each at most once
  std::vector<uint8_t> role((size_t)V, 0);
  for (int32_t i = 0; i < k; i++) {
    if (sources[i] < 0 || sources[i] >= V || sinks[i] < 0 || sinks[i] >= V) return fail(WBPR_EINVAL, "terminal out of range");
    if (role[sources[i]]) return fail(WBPR_EINVAL, "a vertex is listed twice as a terminal");
    role[sources[i]] = 1;
  }
  for (int32_t i = 0; i < k; i++) {
    if (role[sinks[i]]) return fail(WBPR_EINVAL, "a vertex is listed twice as a terminal");
    role[sinks[i]] = 2;
  }
  // super-arcs: S -> source with the source's outgoing capacity, sink -> T
  // with the sink's incoming capacity; neither can bind, and both must fit int32
  std::vector<int64_t> out_cap((size_t)V, 0), in_cap((size_t)V, 0);
  for (int32_t u = 0; u < V; u++)
    for (int64_t a = g->row_ptr[u]; a < g->row_ptr[u + 1]; a++) {
      if (g->cap[a] < 0) return fail(WBPR_EINVAL, "negative capacity");
      if (g->col[a] == u) continue;
      out_cap[u] += g->cap[a];
      in_cap[g->col[a]] += g->cap[a];
    }
  for (int32_t v = 0; v < V; v++)
    if ((role[v] == 1 && out_cap[v] > 0x7fffffffll) || (role[v] == 2 && in_cap[v] > 0x7fffffffll))
      return fail(WBPR_EOVERFLOW, "a terminal's capacity sum exceeds int32");
  // augmented CSR: rows 0..V-1 keep their arcs (a sink's row gains a last
  // arc to T = V + 1, the largest id, so sorted rows stay sorted); row S = V
  // lists the sources in increasing id; row T is empty
  const int32_t S = V, T = V + 1, V2 = V + 2;
  const int64_t E2 = E + 2 * (int64_t)k;
  std::vector<int64_t> rp2((size_t)V2 + 1);
  std::vector<int32_t> col2((size_t)E2), cap2((size_t)E2);
  int64_t p = 0;
  for (int32_t u = 0; u < V; u++) {
    rp2[u] = p;
    for (int64_t a = g->row_ptr[u]; a < g->row_ptr[u + 1]; a++, p++) {
      col2[p] = g->col[a];
      cap2[p] = g->cap[a];
    }
    if (role[u] == 2) {
      col2[p] = T;
      cap2[p] = (int32_t)in_cap[u];
      p++;
    }
  }
  rp2[S] = p;
  for (int32_t v = 0; v < V; v++)
    if (role[v] == 1) {
      col2[p] = v;
      cap2[p] = (int32_t)out_cap[v];
      p++;
    }
  rp2[T] = p;
  rp2[V2] = p;
  wbpr_csr g2{V2, E2, rp2.data(), col2.data(), cap2.data()};
  std::vector<int32_t> flow2(arc_flow ? (size_t)E2 : 0);
  std::vector<uint8_t> side2(cut_side ? (size_t)V2 : 0);
  rc = wbpr_solve(c, &g2, S, T, value, arc_flow ? flow2.data() : nullptr, cut_side ? side2.data() : nullptr, stats);
  if (rc) return rc;
  if (arc_flow)
    for (int32_t u = 0; u < V; u++) {
      const int64_t n = g->row_ptr[u + 1] - g->row_ptr[u];
      if (n > 0) std::memcpy(arc_flow + g->row_ptr[u], flow2.data() + rp2[u], 4 * (size_t)n);
    }
  if (cut_side) std::memcpy(cut_side, side2.data(), (size_t)V);
  return WBPR_OK;
}

}  // extern "C"
