// Residual-graph builder: CSR of input arcs -> bidirectional CSR (paper,
// section 3.2).  Each row u holds one entry per distinct neighbour v that is
// joined to u by an arc in either direction, columns ascending.  Parallel and
// antiparallel input arcs are merged: entry (u,v) starts with residual
// sum c(u->v) and its mate (v,u) with sum c(v->u).  The paper finds the mate
// by binary search in row v; here the builder records it once in rev[]
// (constant-time mate access, paid for with 4 bytes per entry).
//
// Pipeline, entirely on the GPU:
//   1. validate + emit two keys per arc: (u,v) forward and (v,u) backward,
//      payload = arc index (forward) or E + arc index (backward); each
//      arc's row from its tile's row starts staged in LDS
//   2. sorted (row, column) sequence of all keys: when every input row lists
//      its columns in non-decreasing order (the common case), the forward
//      keys are sorted already and the backward keys need only a stable sort
//      on their row (the head of the arc), then the two are merged; else a
//      stable radix sort of all keys on (row, column), self-loops last
//   3. group heads -> unique entry ids (scan); each head walks its group
//      for the merged capacity and the parallel-arc prefixes (long groups:
//      one workgroup each).  On the sorted path, when no row repeats a
//      column more than MT_RUN times, steps 2 (the merge) and 3 are one
//      kernel with a decoupled look-back over tiles (k_merge_entries)
//   4. row pointers, mates and arc->entry map, parallel-arc prefixes; the
//      pairwise int32 overflow check runs only if some entry holds >= 2^30
#include "wb_common.h"
#include "wb_internal.h"
#include "wb_kernels.h"

namespace wb {

static int bits_for(int64_t n) {
  int b = 1;
  while ((1ll << b) < n) b++;
  return b;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

namespace {
struct Scratch {
  uint64_t *k0, *k1;
  uint32_t *v0, *v1;
  int32_t *head, *hx, *uid_of, *gstart, *rowcnt, *rptr, *hist, *stemp;  // gstart: long-group list
};

size_t carve_scratch(int32_t V, int64_t E, void *mem, Scratch *s) {
  int64_t N = 2 * E > 0 ? 2 * E : 1;
  int64_t hn = radix_hist_elems(N);
  int64_t st = scan_temp_elems(hn > N + 1 ? hn : (N + 1 > V + 1 ? N + 1 : V + 1)) + 2;
  char *base = (char *)mem, *p = base;
  auto take = [&](size_t bytes) { char *q = p; p += align256(bytes); return (void *)q; };
  s->k0 = (uint64_t *)take(8 * N);
  s->k1 = (uint64_t *)take(8 * N);
  s->v0 = (uint32_t *)take(4 * N);
  s->v1 = (uint32_t *)take(4 * N);
  s->head = (int32_t *)take(4 * N);
  s->hx = (int32_t *)take(4 * N);
  s->uid_of = (int32_t *)take(4 * N);
  s->gstart = (int32_t *)take(4 * (N + 1));
  s->rowcnt = (int32_t *)take(4 * ((size_t)V + 1));
  s->rptr = (int32_t *)take(4 * ((size_t)V + 1));
  s->hist = (int32_t *)take(4 * (size_t)hn);
  s->stemp = (int32_t *)take(4 * (size_t)st);
  return (size_t)(p - base);
}
}  // namespace

size_t build_scratch_bytes(int32_t V, int64_t E) {
  Scratch s;
  return carve_scratch(V, E, nullptr, &s) + 256;
}

constexpr int BT = 256;

static unsigned grid_for(int64_t n, int per_block = BT) {
  int64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

__global__ void k_check_rowptr(const int64_t *rp, int32_t V, int64_t E, BuildStatus *st, int32_t *rowcnt) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= V; v += (int64_t)gridDim.x * blockDim.x) {
    rowcnt[v] = 0;
    if (v == 0 && rp[0] != 0) atomicAdd(&st->bad_input, 1);
    if (v == V && rp[V] != E) atomicAdd(&st->bad_input, 1);
    if (v < V && rp[v + 1] < rp[v]) atomicAdd(&st->bad_input, 1);
  }
}

// Sum (MAX false) or maximum over the workgroup, returned in thread 0.
// Every thread of the workgroup calls it; blockDim.x <= BT.
template <bool MAX>
__device__ int block_reduce_i32(int x) {
  __shared__ int s_part[BT / WB_WAVE];
#pragma unroll
  for (int o = WB_WAVE / 2; o > 0; o >>= 1) {
    const int y = __shfl_xor(x, o, WB_WAVE);
    x = MAX ? max(x, y) : x + y;
  }
  __syncthreads();  // a previous call may still read s_part
  if (lane() == 0) s_part[threadIdx.x / WB_WAVE] = x;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int w = 1; w < (int)(blockDim.x / WB_WAVE); w++) x = MAX ? max(x, s_part[w]) : x + s_part[w];
  return x;
}

// Step 1a (RCSR).  Row of every arc without a per-arc search: cnt[rp[u]] += 1 for
// each row u >= 1 that starts inside [0, E); the inclusive prefix sum of cnt
// at arc i then counts the rows u >= 1 that start at or before i, which is
// the row of i (empty rows share a start and are counted, so the last of
// them wins, as it must).  The count stays below V whatever rp holds.
__global__ void k_row_marks(const int64_t *rp, int32_t V, int64_t E, int32_t *cnt) {
  for (int64_t u = 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < V; u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = rp[u];
    if (p >= 0 && p < E) atomicAdd(&cnt[p], 1);
  }
}

// Longest run of equal columns in a sorted row that the fused merge below
// accepts; a group of equal keys then holds at most 2 * MT_RUN items.
constexpr int MT_RUN = 256;

// Step 1 (BCSR).  Forward key (u,v) goes to fkeys[i], backward key (v,u)
// to bkeys[i], with u the row of arc i; a self-loop (or an out-of-range
// column, dropped as one) gets (u,u) in both, which keeps a column-sorted
// row sorted; the full-sort path turns them into the largest key.  Also
// checks that every row's columns are non-decreasing and whether a row
// repeats a column more than MT_RUN times.  Counters are reduced per
// workgroup, one atomic per workgroup and status word.  The rows come
// without a per-arc array: arcs are taken in tiles of EK_TILE, k_tile_rows
// gives each tile the rows of its first and last arcs (one binary search
// over row_ptr per tile bound), the tile loads those rows' starts into LDS,
// and each arc finds its row there by a short binary search (marks at the
// row starts and a prefix sum over all arcs, as the RCSR builder does, cost
// a fill, three scan passes and the array).
constexpr int EK_TILE = 2048;
constexpr int EK_ROWS = 2048;  // row starts a tile keeps in LDS; more: searched in row_ptr

// Largest row r in [lo, hi] with rp[r] <= i (rp non-decreasing; clamped).
__device__ __forceinline__ int32_t row_search(const int64_t *rp, int32_t lo, int32_t hi, int64_t i) {
  while (lo < hi) {
    const int32_t m = lo + (hi - lo + 1) / 2;
    if (rp[m] <= i) lo = m; else hi = m - 1;
  }
  return lo;
}

__global__ void k_tile_rows(const int64_t *rp, int32_t V, int64_t E, int64_t ntiles, int32_t *trow) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= ntiles; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x < ntiles ? x * EK_TILE : E - 1;  // tile starts, then the last arc
    trow[x] = row_search(rp, 0, V - 1, i);
  }
}

// Payloads of the forward keys (their arc indices), for the paths that
// carry them through a merge or sort; the fused merge knows them by position.
__global__ void k_iota(uint32_t *v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(BT) k_emit_keys_tiled(const int64_t *rp, const int32_t *trow, int64_t ntiles,
                                                        const int32_t *col, const int32_t *cap, int32_t V, int64_t E,
                                                        int vb, uint64_t *fkeys, uint64_t *bkeys,
                                                        uint32_t *bvals, int32_t *arc2ent, int32_t *acap,
                                                        int32_t *hist, BuildStatus *st) {
  static_assert(RADIX_TILE % EK_TILE == 0, "a radix tile is whole emission tiles");
  constexpr int EK_PER_RS = RADIX_TILE / EK_TILE;
  constexpr int NDIG = 1 << RADIX_BITS;
  __shared__ int64_t s_rp[EK_ROWS];
  __shared__ int s_dig[NDIG];
  int nself = 0, bad = 0, unsorted = 0, longrun = 0;
  // a workgroup takes the emission tiles of one radix tile at a time and
  // counts the first digit of their backward keys (the low RADIX_BITS bits
  // of the row) for the radix sort's first pass
  const int64_t ngroups = (ntiles + EK_PER_RS - 1) / EK_PER_RS;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {  // workgroup-uniform
    for (int d = threadIdx.x; d < NDIG; d += BT) s_dig[d] = 0;  // ordered before the counts by the tile's barriers
    const int64_t tend = (grp + 1) * EK_PER_RS < ntiles ? (grp + 1) * EK_PER_RS : ntiles;
    for (int64_t t = grp * EK_PER_RS; t < tend; t++) {  // workgroup-uniform
      const int64_t a0 = t * EK_TILE;
      const int64_t a1 = a0 + EK_TILE < E ? a0 + EK_TILE : E;
      const int32_t r0 = trow[t];
      const int32_t r1 = t + 1 < ntiles ? trow[t + 1] : trow[ntiles];  // row of a1 (or of the last arc)
      const int32_t lo = r0 < r1 ? r0 : r1, hi = r0 < r1 ? r1 : r0;  // ordered even for a malformed row_ptr
      const bool in_lds = hi - lo + 1 <= EK_ROWS;
      __syncthreads();  // s_rp of the previous tile is read
      if (in_lds)
        for (int32_t r = lo + threadIdx.x; r <= hi; r += BT) s_rp[r - lo] = rp[r];
      __syncthreads();
      for (int64_t i = a0 + threadIdx.x; i < a1; i += BT) {
        int32_t r;
        if (in_lds) {
          int32_t l = 0, h = hi - lo;  // largest index with s_rp <= i
          while (l < h) {
            const int32_t m = l + (h - l + 1) / 2;
            if (s_rp[m] <= i) l = m; else h = m - 1;
          }
          r = lo + l;
        } else {
          r = row_search(rp, lo, hi, i);
        }
        const uint64_t u = (uint64_t)r;
        const int32_t vv = col[i];
        const int32_t c = cap[i];
        const bool ok = vv >= 0 && vv < V;
        if (!ok || c < 0) bad++;
        const int64_t rs = in_lds ? s_rp[r - lo] : rp[r];
        if (i > rs && col[i - 1] > vv) unsorted++;
        if (i - MT_RUN >= rs && i >= MT_RUN && col[i - MT_RUN] == vv) longrun++;
        const uint64_t v = ok ? (uint64_t)vv : u;
        if (u == v) nself++;
        fkeys[i] = (u << vb) | v;
        bkeys[i] = (v << vb) | u;
        arc2ent[i] = u == v ? -1 : 0;
        bvals[i] = (uint32_t)(E + i);
        acap[i] = c;
        atomicAdd(&s_dig[(int)(v & (NDIG - 1))], 1);
      }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < NDIG; d += BT) hist[(int64_t)d * ngroups + grp] = s_dig[d];
    __syncthreads();  // the counts are read before the next group clears them
  }
  nself = block_reduce_i32<false>(nself);
  bad = block_reduce_i32<false>(bad);
  unsorted = block_reduce_i32<false>(unsorted);
  longrun = block_reduce_i32<false>(longrun);
  if (threadIdx.x == 0) {
    if (nself) atomicAdd(&st->nself, nself);
    if (bad) atomicAdd(&st->bad_input, bad);
    if (unsorted) atomicAdd(&st->unsorted, unsorted);
    if (longrun) atomicAdd(&st->longrun, longrun);
  }
}

// Full-sort path: self-loop keys (u,u) become the largest key, so the sort
// puts them last where the later steps drop them.
__global__ void k_selfloops_last(uint64_t *keys, int64_t N, int vb) {
  const uint64_t ALL = (vb * 2 >= 64) ? ~0ull : ((1ull << (2 * vb)) - 1);
  const uint64_t cmask = (1ull << vb) - 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    if ((k >> vb) == (k & cmask)) keys[i] = ALL;
  }
}

// Sorted-rows path: merge two sorted runs a [0, n) and b [0, n) into out
// (merge path; equal keys take a first).  A workgroup makes MERGE_TILE
// outputs: two threads find the tile's split of a and b by a binary search
// along its first and last diagonal, the workgroup stages both input ranges
// in LDS (coalesced), and each thread finds its own MERGE_ITEMS outputs by a
// short search in LDS and records where each comes from; the workgroup then
// writes the tile out in order (coalesced).
constexpr int MERGE_THREADS = 256;
constexpr int MERGE_ITEMS = 8;
constexpr int MERGE_TILE = MERGE_THREADS * MERGE_ITEMS;

// smallest i in [max(0, d - nb), min(d, na)] with a[i] > b[d - i - 1]
template <typename K>
__device__ __forceinline__ int64_t merge_split(const K *a, int64_t na, const K *b, int64_t nb, int64_t d) {
  int64_t lo = d > nb ? d - nb : 0, hi = d < na ? d : na;
  while (lo < hi) {
    const int64_t i = (lo + hi) >> 1;
    if (a[i] <= b[d - i - 1]) lo = i + 1; else hi = i;
  }
  return lo;
}

// Self-loop items: after the full sort they are the last 2 nself items
// (dropped by mraw); on the sorted-rows path they stay inline with key (u,u)
// and every step skips them.
__device__ __forceinline__ bool self_key(uint64_t k, int vb) { return (k >> vb) == (k & ((1ull << vb) - 1)); }

// The merge also marks where each group of equal keys starts (head[o] = 1
// unless the key is a self-loop's): the output before the tile's first one
// is the larger of the two inputs' predecessors.
__global__ void __launch_bounds__(MERGE_THREADS) k_merge(const uint64_t *ka, const uint32_t *va, const uint64_t *kb,
                                                         const uint32_t *vb, int64_t n, uint64_t *ko, uint32_t *vo,
                                                         int32_t *head, int kbits) {
  __shared__ uint64_t s_k[MERGE_TILE];
  __shared__ uint32_t s_v[MERGE_TILE];
  __shared__ uint16_t s_src[MERGE_TILE];
  __shared__ int64_t s_split[2];
  static_assert(MERGE_TILE <= 65536, "LDS source index is 16-bit");
  const int64_t total = 2 * n;
  for (int64_t d0 = (int64_t)blockIdx.x * MERGE_TILE; d0 < total; d0 += (int64_t)gridDim.x * MERGE_TILE) {
    const int64_t d1 = d0 + MERGE_TILE < total ? d0 + MERGE_TILE : total;
    if (threadIdx.x < 2) s_split[threadIdx.x] = merge_split(ka, n, kb, n, threadIdx.x == 0 ? d0 : d1);
    __syncthreads();
    const int64_t i0 = s_split[0], i1 = s_split[1];
    const int na = (int)(i1 - i0), nb = (int)((d1 - i1) - (d0 - i0));
    const int64_t j0 = d0 - i0;
    for (int x = threadIdx.x; x < na + nb; x += MERGE_THREADS) {
      if (x < na) {
        s_k[x] = ka[i0 + x];
        s_v[x] = va[i0 + x];
      } else {
        s_k[x] = kb[j0 + x - na];
        s_v[x] = vb[j0 + x - na];
      }
    }
    __syncthreads();
    const int dl = threadIdx.x * MERGE_ITEMS;
    if (dl < na + nb) {
      const uint64_t *A = s_k, *B = s_k + na;
      int i = (int)merge_split(A, na, B, nb, dl), j = dl - i;
      const int end = dl + MERGE_ITEMS < na + nb ? dl + MERGE_ITEMS : na + nb;
      for (int o = dl; o < end; o++) {
        const bool take_a = j >= nb || (i < na && A[i] <= B[j]);
        s_src[o] = (uint16_t)(take_a ? i++ : na + j++);
      }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < na + nb; x += MERGE_THREADS) {
      const int src = s_src[x];
      const uint64_t k = s_k[src];
      ko[d0 + x] = k;
      vo[d0 + x] = s_v[src];
      bool first;
      if (x > 0) {
        first = s_k[s_src[x - 1]] != k;
      } else if (d0 == 0) {
        first = true;
      } else {
        const uint64_t pa = i0 > 0 ? ka[i0 - 1] : 0, pb = j0 > 0 ? kb[j0 - 1] : 0;
        first = (pa > pb ? pa : pb) != k;
      }
      head[d0 + x] = first && !self_key(k, kbits) ? 1 : 0;
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

// Step 3a.  head[i] = 1 where a new (row, column) group starts.
__global__ void k_heads(const uint64_t *keys, int64_t N, int vb, bool inline_self, const BuildStatus *st,
                        int32_t *head) {
  int64_t mraw = inline_self ? N : N - 2 * (int64_t)st->nself;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
    head[i] = (i < mraw && (i == 0 || keys[i] != keys[i - 1]) && !(inline_self && self_key(keys[i], vb))) ? 1 : 0;
  }
}

// Step 3b.  A group (a run of equal keys: the forward items of every arc
// u->v and the backward items of every arc v->u) becomes entry hx[head].
// Its head walks it in sorted order (the sort is stable, so a group's arcs
// are in input order), records the entry id of every item under its payload,
// the capacity of earlier parallel arcs for each forward arc, and writes the
// entry: column and summed forward capacity, plus the initial residual copy.
// A sum above INT32_MAX is an overflow by itself; sums of at least 2^30 are
// counted, since only such an entry can overflow together with its mate (two
// sums below 2^30 add up to less than 2^31).  Groups longer than GROUP_WALK
// items (many parallel arcs) are listed for k_long_groups instead, so no
// thread walks far.
constexpr int GROUP_WALK = 256;

__device__ __forceinline__ void write_entry(int32_t u, uint64_t key, uint64_t cmask, int32_t vbase, long long c,
                                            int2 *ent, int32_t *cap0, int *big, int *ovf) {
  *big += c >= (1ll << 30);
  *ovf += c > 0x7fffffffll;
  const int32_t c32 = c > 0x7fffffffll ? 0 : (int32_t)c;
  ent[u] = make_int2(vbase + (int)(key & cmask), c32);
  cap0[u] = c32;
}

// Sorted-rows path, fused (no row repeats a column more than MT_RUN times):
// the merged keys, the head flags and their prefix sum never go through
// memory.  The merge is cut into tiles of about MT_TILE outputs whose bounds
// are moved forward past the group of equal keys that straddles them (a
// group holds at most MT_SLACK items, so a tile holds fewer than MT_CAP),
// which puts every group inside one tile.  Three passes: the tile bounds
// (k_merge_splits), the number of entries (group heads) of every tile
// (k_merge_count) and their prefix sum, then the entries (k_merge_entries):
// each workgroup merges its tile in LDS, every item records its entry id
// under its payload, every forward item the capacity of the earlier
// parallel arcs of its group (a segmented prefix sum over the workgroup),
// and the group ends write the entries (column, summed capacity, row).
// (A single pass with a decoupled look-back between tiles was slower: its
// waits held back the scattered writes.)
constexpr int MT_THREADS = 256;
constexpr int MT_TILE = 2048;
constexpr int MT_SLACK = 2 * MT_RUN;
constexpr int MT_CAP = MT_TILE + MT_SLACK;
constexpr int MT_ITEMS = MT_CAP / MT_THREADS;
constexpr int MT_WAVES = MT_THREADS / WB_WAVE;
static_assert(MT_CAP % MT_THREADS == 0, "tile capacity is a whole number of items per thread");
static_assert(MT_CAP <= 65536, "LDS source index is 16-bit");

// First index in [lo, min(lo + MT_SLACK, n)) whose key exceeds k, else that bound.
__device__ __forceinline__ int64_t run_end(const uint64_t *x, int64_t lo, int64_t n, uint64_t k) {
  int64_t hi = lo + MT_SLACK < n ? lo + MT_SLACK : n;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (x[m] <= k) lo = m + 1; else hi = m;
  }
  return lo;
}

// Merge-path split of a and b (n keys each) at output d, moved forward past
// the group of equal keys that straddles d.  *bad is set if that group is
// longer than MT_SLACK (the long-run check rules this out).
__device__ void mt_split(const uint64_t *a, const uint64_t *b, int64_t n, int64_t d, int64_t *ia, int64_t *jb,
                         int *bad) {
  int64_t i = merge_split(a, n, b, n, d), j = d - i;
  if (d > 0 && d < 2 * n) {
    const uint64_t pa = i > 0 ? a[i - 1] : 0, pb = j > 0 ? b[j - 1] : 0;
    const uint64_t pk = pa > pb ? pa : pb;  // last output before d
    const uint64_t nk = (i < n && (j >= n || a[i] <= b[j])) ? a[i] : b[j];  // output d
    if (nk == pk) {
      const int64_t i2 = run_end(a, i, n, pk), j2 = run_end(b, j, n, pk);
      if ((i2 - i) + (j2 - j) >= MT_SLACK) *bad = 1;
      i = i2;
      j = j2;
    }
  }
  *ia = i;
  *jb = j;
}

// Tile bounds, one thread per bound: split[2x], split[2x+1] = positions in
// a and b where tile x starts.
__global__ void k_merge_splits(const uint64_t *a, const uint64_t *b, int64_t n, int64_t ntiles, int64_t *split,
                               BuildStatus *st) {
  int bad = 0;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= ntiles; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = x * MT_TILE < 2 * n ? x * MT_TILE : 2 * n;
    int64_t i, j;
    mt_split(a, b, n, d, &i, &j, &bad);
    split[2 * x] = i;
    split[2 * x + 1] = j;
  }
  if (bad) atomicAdd(&st->bad_input, 1);
}

// Tile t's item counts (na, nb) from its bounds; false (and counts 0) for a
// tile whose bounds a bad split left out of shape, which k_merge_splits has
// reported.
__device__ __forceinline__ bool mt_tile(const int64_t *split, int64_t t, int64_t *i0, int64_t *j0, int *na, int *nb) {
  *i0 = split[2 * t];
  *j0 = split[2 * t + 1];
  const int64_t a = split[2 * t + 2] - *i0, b = split[2 * t + 3] - *j0;
  const bool ok = a >= 0 && b >= 0 && a + b <= MT_CAP;
  *na = ok ? (int)a : 0;
  *nb = ok ? (int)b : 0;
  return ok;
}

// Entries of every tile: its distinct keys that are not self-loops.  A key
// of the tile's a-range counts at its first occurrence; one of the b-range
// at its first occurrence unless the a-range holds it too (binary search in
// LDS).  Groups do not straddle tiles, so these are the tile's group heads.
__global__ void __launch_bounds__(MT_THREADS) k_merge_count(const uint64_t *ka, const uint64_t *kb, int kbits,
                                                            int64_t ntiles, const int64_t *split, int32_t *heads) {
  __shared__ uint64_t s_k[MT_CAP];
  __shared__ int s_w[MT_WAVES];
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {  // workgroup-uniform
    int64_t i0, j0;
    int na, nb;
    mt_tile(split, t, &i0, &j0, &na, &nb);
    const int cnt = na + nb;  // <= MT_CAP = MT_ITEMS * MT_THREADS
    {
      // every load of the thread is issued before the first LDS store
      uint64_t r[MT_ITEMS];
#pragma unroll
      for (int q = 0; q < MT_ITEMS; q++) {
        const int x = threadIdx.x + q * MT_THREADS;
        r[q] = x < na ? ka[i0 + x] : x < cnt ? kb[j0 + x - na] : 0;
      }
#pragma unroll
      for (int q = 0; q < MT_ITEMS; q++) {
        const int x = threadIdx.x + q * MT_THREADS;
        if (x < cnt) s_k[x] = r[q];
      }
    }
    __syncthreads();
    int h = 0;
    for (int x = threadIdx.x; x < cnt; x += MT_THREADS) {
      const uint64_t k = s_k[x];
      if (self_key(k, kbits)) continue;
      if (x < na) {
        h += x == 0 || s_k[x - 1] != k;
      } else if (x == na || s_k[x - 1] != k) {
        int lo = 0, hi = na;  // first a-item >= k
        while (lo < hi) {
          const int m = (lo + hi) >> 1;
          if (s_k[m] < k) lo = m + 1; else hi = m;
        }
        h += lo == na || s_k[lo] != k;
      }
    }
    h = wave_sum_i32(h);
    if (lane() == 0) s_w[threadIdx.x / WB_WAVE] = h;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < MT_WAVES; w++) tot += s_w[w];
      heads[t] = tot;
    }
    __syncthreads();  // LDS is reused by the next tile
  }
}

__global__ void __launch_bounds__(MT_THREADS)
    k_merge_entries(const uint64_t *ka, const uint64_t *kb, const uint32_t *vb, int64_t n, int kbits,
                    const int32_t *cap, int32_t vbase, int64_t ntiles, const int64_t *split, const int32_t *hpre,
                    BuildStatus *st, int2 *ent, int32_t *cap0, int32_t *erow, int32_t *uid_of, int32_t *pbefore_arc) {
  // a-items (forward arcs, payload = their index) keep their capacity in
  // s_v, b-items (backward) their payload; both arrays are reused to stage
  // the outputs so that they leave in coalesced runs
  __shared__ uint64_t s_k[MT_CAP];
  __shared__ uint32_t s_v[MT_CAP];
  __shared__ uint16_t s_src[MT_CAP];
  __shared__ int s_wh[MT_WAVES];
  __shared__ int s_wf[MT_WAVES];
  __shared__ long long s_ws[MT_WAVES];
  const uint64_t cmask = (1ull << kbits) - 1;
  const int64_t total = 2 * n;
  const int w = threadIdx.x / WB_WAVE;
  int big = 0, ovf = 0;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {  // workgroup-uniform
    int64_t i0, j0;
    int na, nb;
    mt_tile(split, t, &i0, &j0, &na, &nb);
    const int cnt = na + nb;
    const long long P = hpre[t];  // entries of the earlier tiles
    {
      // every load of the thread is issued before the first LDS store
      uint64_t r[MT_ITEMS];
      uint32_t rv[MT_ITEMS];
#pragma unroll
      for (int q = 0; q < MT_ITEMS; q++) {
        const int x = threadIdx.x + q * MT_THREADS;
        r[q] = 0;
        rv[q] = 0;
        if (x < na) {
          r[q] = ka[i0 + x];
          rv[q] = (uint32_t)cap[i0 + x];
        } else if (x < cnt) {
          r[q] = kb[j0 + x - na];
          rv[q] = vb[j0 + x - na];
        }
      }
#pragma unroll
      for (int q = 0; q < MT_ITEMS; q++) {
        const int x = threadIdx.x + q * MT_THREADS;
        if (x < cnt) {
          s_k[x] = r[q];
          s_v[x] = rv[q];
        }
      }
    }
    __syncthreads();
    const int x0 = threadIdx.x * MT_ITEMS;
    if (x0 < cnt) {
      const uint64_t *A = s_k, *B = s_k + na;
      int i = (int)merge_split(A, na, B, nb, x0), j = x0 - i;
      const int end = x0 + MT_ITEMS < cnt ? x0 + MT_ITEMS : cnt;
      for (int o = x0; o < end; o++) {
        const bool take_a = j >= nb || (i < na && A[i] <= B[j]);
        s_src[o] = (uint16_t)(take_a ? i++ : na + j++);
      }
    }
    __syncthreads();
    // this thread's MT_ITEMS consecutive outputs: keys, payloads, forward
    // capacities; group starts (seg), self-loop items, group ends
    uint64_t kk[MT_ITEMS];
    uint32_t pv[MT_ITEMS];
    int32_t cv[MT_ITEMS];
    unsigned segm = 0, selfm = 0, endm = 0;
    uint64_t prev = x0 > 0 && x0 <= cnt ? s_k[s_src[x0 - 1]] : 0;
    // key after this thread's last output (ends the thread's last group or not)
    const uint64_t after = x0 + MT_ITEMS < cnt ? s_k[s_src[x0 + MT_ITEMS]] : 0;
#pragma unroll
    for (int q = 0; q < MT_ITEMS; q++) {
      const int x = x0 + q;
      kk[q] = 0;
      pv[q] = 0;
      cv[q] = 0;
      if (x < cnt) {
        const int src = s_src[x];
        kk[q] = s_k[src];
        const bool sf = self_key(kk[q], kbits);
        if (src < na) {
          pv[q] = (uint32_t)(i0 + src);
          cv[q] = sf ? 0 : (int32_t)s_v[src];
        } else {
          pv[q] = s_v[src];
        }
        if (x == 0 || kk[q] != prev) segm |= 1u << q;
        if (sf) selfm |= 1u << q;
        prev = kk[q];
      }
    }
#pragma unroll
    for (int q = 0; q < MT_ITEMS; q++) {
      const int x = x0 + q;
      const bool nseg = q + 1 < MT_ITEMS ? ((segm >> (q + 1)) & 1) != 0 : after != kk[q];
      if (x < cnt && (x + 1 >= cnt || nseg)) endm |= 1u << q;
    }
    int nh = 0;
    long long tail = 0;
#pragma unroll
    for (int q = 0; q < MT_ITEMS; q++) {
      const bool seg = (segm >> q) & 1;
      nh += seg && !((selfm >> q) & 1);
      if (seg) tail = 0;
      tail += cv[q];
    }
    const int fl = segm != 0;
    // workgroup scans: heads (sum) and the group sums carried into each
    // thread (segmented: a thread with a group start resets the carry)
    int hin = nh, fin = fl;
    long long sin = tail;
#pragma unroll
    for (int d = 1; d < WB_WAVE; d <<= 1) {
      const int hy = __shfl_up(hin, d, WB_WAVE);
      const int fy = __shfl_up(fin, d, WB_WAVE);
      const long long sy = (long long)shfl_up_u64((unsigned long long)sin, d);
      if (lane() >= d) {
        hin += hy;
        sin = fin ? sin : sy + sin;
        fin |= fy;
      }
    }
    if (lane() == WB_WAVE - 1) {
      s_wh[w] = hin;
      s_wf[w] = fin;
      s_ws[w] = sin;
    }
    __syncthreads();
    int hoff = 0, H = 0;  // heads before this thread in the tile, in the tile
    long long cs = 0;     // carry from the earlier waves
#pragma unroll
    for (int ww = 0; ww < MT_WAVES; ww++) {
      if (ww < w) {
        hoff += s_wh[ww];
        cs = s_wf[ww] ? s_ws[ww] : cs + s_ws[ww];
      }
      H += s_wh[ww];
    }
    {
      // exclusive within the wave: the inclusive value of the lane before
      const int hx = __shfl_up(hin, 1, WB_WAVE);
      const int fx = __shfl_up(fin, 1, WB_WAVE);
      const long long sx = (long long)shfl_up_u64((unsigned long long)sin, 1);
      if (lane() > 0) {
        hoff += hx;
        cs = fx ? sx : cs + sx;
      }
    }
    __syncthreads();  // the items are in registers: LDS is free
    // entry ids and earlier-parallel-arc capacities, staged by output
    // position: s_k[x] = uid << 32 | payload (uid ~0: self-loop), s_v[x] =
    // capacity before the item in its group; group totals stay in registers
    long long run = cs;
    int32_t hid = (int32_t)(P + hoff);  // entries before this thread's first output
    int32_t gtot[MT_ITEMS];  // group total (clipped as stored), -1: not a group end
    int32_t gent[MT_ITEMS];
#pragma unroll
    for (int q = 0; q < MT_ITEMS; q++) {
      const int x = x0 + q;
      gtot[q] = -1;
      gent[q] = 0;
      if (x < cnt) {
        const bool seg = (segm >> q) & 1, self = (selfm >> q) & 1;
        if (seg) run = 0;
        const long long before = run;
        run += cv[q];
        if (seg && !self) hid++;
        const uint32_t u = self ? 0xffffffffu : (uint32_t)(hid - 1);
        s_k[x] = ((unsigned long long)u << 32) | pv[q];
        s_v[x] = (uint32_t)(before > 0x7fffffffll ? 0 : before);
        if (!self && ((endm >> q) & 1)) {
          big += run >= (1ll << 30);
          ovf += run > 0x7fffffffll;
          gtot[q] = run > 0x7fffffffll ? 0 : (int32_t)run;
          gent[q] = hid - 1;
        }
      }
    }
    __syncthreads();
    for (int x = threadIdx.x; x < cnt; x += MT_THREADS) {
      const unsigned long long r = s_k[x];
      const uint32_t u = (uint32_t)(r >> 32), pl = (uint32_t)r;
      if (u != 0xffffffffu && u < (uint64_t)total) {  // always in range; guards the writes
        uid_of[pl] = (int32_t)u;
        if (pl < (uint64_t)n) pbefore_arc[pl] = (int32_t)s_v[x];
      }
    }
    __syncthreads();
    // entries P .. P + H - 1 belong to this tile's group ends, in order:
    // stage key and total by entry, then write the entries out
#pragma unroll
    for (int q = 0; q < MT_ITEMS; q++) {
      if (gtot[q] >= 0) {
        const long long h = (long long)gent[q] - P;
        if (h >= 0 && h < MT_CAP) {  // always
          s_k[h] = kk[q];
          s_v[h] = (uint32_t)gtot[q];
        }
      }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < H && h < MT_CAP; h += MT_THREADS) {
      const int64_t u = P + h;
      if (u < total) {
        const uint64_t key = s_k[h];
        const int32_t c32 = (int32_t)s_v[h];
        ent[u] = make_int2(vbase + (int)(key & cmask), c32);
        cap0[u] = c32;
        erow[u] = (int32_t)(key >> kbits);
      }
    }
    __syncthreads();  // LDS is reused by the next tile
  }
  big = block_reduce_i32<false>(big);
  ovf = block_reduce_i32<false>(ovf);
  if (threadIdx.x == 0) {
    if (big) atomicAdd(&st->big, big);
    if (ovf) atomicAdd(&st->overflow, ovf);
  }
}

// Row pointers of the fused path: rptr[x] = first entry whose row is >= x
// (entries are in row order and erow[] holds each one's row).
__global__ void k_rowptr_rows(const int32_t *erow, int32_t V, const BuildStatus *st, int32_t *rptr) {
  const int32_t M = st->M;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= V; x += (int64_t)gridDim.x * blockDim.x) {
    int32_t lo = 0, hi = M;
    while (lo < hi) {
      const int32_t mid = lo + (hi - lo) / 2;
      if (erow[mid] < x) lo = mid + 1; else hi = mid;
    }
    rptr[x] = lo;
  }
}

__global__ void k_groups(const uint64_t *keys, const uint32_t *vals, int64_t N, int vb, bool inline_self,
                         const int32_t *cap, BuildStatus *st, const int32_t *head, const int32_t *hx, int32_t vbase,
                         int2 *ent, int32_t *cap0, int32_t *uid_of, int32_t *pbefore_arc, int32_t *long_list) {
  const int64_t mraw = inline_self ? N : N - 2 * (int64_t)st->nself;
  const uint32_t E = (uint32_t)(N / 2);  // payloads below E are forward arcs
  const uint64_t cmask = (1ull << vb) - 1;
  int big = 0, ovf = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < mraw; i += (int64_t)gridDim.x * blockDim.x) {
    if (!head[i]) continue;  // also every self-loop key
    const uint64_t key = keys[i];
    const int32_t u = hx[i];
    long long acc = 0;
    int64_t j = i;
    for (; j < mraw && j - i < GROUP_WALK && keys[j] == key; j++) {
      const uint32_t pl = vals[j];
      uid_of[pl] = u;
      if (pl < E) {
        pbefore_arc[pl] = acc > 0x7fffffffll ? 0 : (int32_t)acc;
        acc += cap[pl];
      }
    }
    if (j - i == GROUP_WALK && j < mraw && keys[j] == key) {
      long_list[atomicAdd(&st->nlong, 1)] = (int32_t)i;  // at most N / GROUP_WALK of them
      continue;
    }
    write_entry(u, key, cmask, vbase, acc, ent, cap0, &big, &ovf);
  }
  big = block_reduce_i32<false>(big);
  ovf = block_reduce_i32<false>(ovf);
  if (threadIdx.x == 0) {
    if (big) atomicAdd(&st->big, big);
    if (ovf) atomicAdd(&st->overflow, ovf);
  }
}

// Exclusive prefix sum over the workgroup (BT threads); total in *total.
__device__ long long block_excl_scan(long long x, long long *total) {
  __shared__ long long s_w[BT / WB_WAVE];
  long long incl = x;
#pragma unroll
  for (int o = 1; o < WB_WAVE; o <<= 1) {
    const unsigned long long y = shfl_u64((unsigned long long)incl, lane() >= o ? lane() - o : lane());
    if (lane() >= o) incl += (long long)y;
  }
  __syncthreads();  // s_w may still be read by a previous call
  if (lane() == WB_WAVE - 1) s_w[threadIdx.x / WB_WAVE] = incl;
  __syncthreads();
  long long before = 0, all = 0;
  for (int w = 0; w < BT / WB_WAVE; w++) {
    if (w < (int)(threadIdx.x / WB_WAVE)) before += s_w[w];
    all += s_w[w];
  }
  *total = all;
  return before + incl - x;
}

// Step 3b'.  Long groups, one workgroup each: tiles of BT items, a block
// prefix sum of the forward capacities, the running total carried over.
__global__ void __launch_bounds__(BT) k_long_groups(const uint64_t *keys, const uint32_t *vals, int64_t N, int vb,
                                                    bool inline_self, const int32_t *cap, BuildStatus *st,
                                                    const int32_t *hx, int32_t vbase, int2 *ent, int32_t *cap0,
                                                    int32_t *uid_of, int32_t *pbefore_arc, const int32_t *long_list) {
  const int64_t mraw = inline_self ? N : N - 2 * (int64_t)st->nself;
  const int32_t nlong = st->nlong;
  const uint32_t E = (uint32_t)(N / 2);
  const uint64_t cmask = (1ull << vb) - 1;
  int big = 0, ovf = 0;
  for (int32_t gi = blockIdx.x; gi < nlong; gi += gridDim.x) {  // workgroup-uniform
    const int64_t i0 = long_list[gi];
    const uint64_t key = keys[i0];
    const int32_t u = hx[i0];
    long long carry = 0;
    for (int64_t base = i0;; base += BT) {
      const int64_t j = base + threadIdx.x;
      const bool in = j < mraw && keys[j] == key;  // the group is one contiguous run
      const uint32_t pl = in ? vals[j] : 0;
      const bool fwd = in && pl < E;
      long long tile = 0;
      const long long pre = block_excl_scan(fwd ? (long long)cap[pl] : 0, &tile);
      if (in) {
        uid_of[pl] = u;
        if (fwd) pbefore_arc[pl] = carry + pre > 0x7fffffffll ? 0 : (int32_t)(carry + pre);
      }
      carry += tile;
      if (__syncthreads_or(!in)) break;
    }
    if (threadIdx.x == 0) write_entry(u, key, cmask, vbase, carry, ent, cap0, &big, &ovf);
  }
  if (threadIdx.x == 0) {
    if (big) atomicAdd(&st->big, big);
    if (ovf) atomicAdd(&st->overflow, ovf);
  }
}

// Step 3c.  Row pointers without atomics (rows such as s and t of a grid cut
// hold millions of entries): rptr[x] = number of merged entries in rows < x
// = number of group heads before the first sorted key of row >= x.
__global__ void k_rowptr(const uint64_t *keys, int64_t N, int vb, bool inline_self, int32_t V, const BuildStatus *st,
                         const int32_t *hx, int32_t *rptr) {
  const int64_t mraw = inline_self ? N : N - 2 * (int64_t)st->nself;
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= V; x += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t target = (uint64_t)x << vb;
    int64_t lo = 0, hi = mraw;  // first position with key >= target
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    rptr[x] = lo < mraw ? hx[lo] : st->M;
  }
}

// Row bounds in the arena: rows of this build start at entry mbase.
__global__ void k_rowb(const int32_t *rptr, int32_t V, int32_t vbase, int32_t mbase, int2 *rowb) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < V; x += (int64_t)gridDim.x * blockDim.x)
    rowb[vbase + x] = make_int2(mbase + rptr[x], mbase + rptr[x + 1]);
}

// Step 4.  Mates and the arc -> entry map (arc order: sequential reads).
// rev and arc2ent point at this build's slices of the arena; the stored
// indices are absolute (local + mbase).
__global__ void k_arcs(int64_t E, const int32_t *uid_of, int32_t mbase, int32_t *rev, int32_t *arc2ent,
                       int32_t *pbefore, BuildStatus *st) {
  const int32_t M = st->M;
  int bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    if (arc2ent[i] < 0) {
      pbefore[i] = 0;
      continue;
    }
    const int32_t f = uid_of[i], b = uid_of[E + i];
    if (f < 0 || f >= M || b < 0 || b >= M) {  // cannot happen unless the build has a bug
      bad++;
      continue;
    }
    rev[f] = mbase + b;
    rev[b] = mbase + f;
    arc2ent[i] = mbase + f;
  }
  bad = block_reduce_i32<false>(bad);
  if (threadIdx.x == 0 && bad) atomicAdd(&st->bad_input, bad);
}

// Step 4b.  Exact pairwise int32 check c(u,v) + c(v,u), needed only when
// some entry holds at least 2^30; otherwise every workgroup leaves at once.
__global__ void k_pair_check(const int32_t *rev, int32_t mbase, const int2 *ent, BuildStatus *st) {
  if (st->big == 0) return;
  const int64_t M = st->M;
  int ovf = 0;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < M; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = rev[j] - mbase;
    if (r < 0 || r >= M) continue;  // k_arcs has reported it
    ovf += (int64_t)ent[j].y + (int64_t)ent[r].y > 0x7fffffffll;
  }
  ovf = block_reduce_i32<false>(ovf);
  if (threadIdx.x == 0 && ovf) atomicAdd(&st->overflow, ovf);
}

// ------------------------------------------------------------------ RCSR
// The paper's other layout (section 3.2, its reversed CSR): no merging.  Row
// x of the arena is x's out-arcs in input order (forward entries, the input
// CSR's own row, shifted by the number of in-arcs of lower vertices), then
// x's in-arcs ordered by tail (reverse entries).  One stable radix sort of
// the arcs by head gives every reverse row and, by binary search over the
// sorted heads, the in-degree prefix R[x]; then
//   first(x) = row_ptr[x] + R[x],   forward entry of arc i = i + R[u],
//   reverse entry of the j-th arc in head order = row_ptr[v + 1] + j.

// Validates arcs and emits the head of every arc as its sort key.
__global__ void k_rc_keys(const int64_t *rp, const int32_t *row_of, const int32_t *col, const int32_t *cap, int32_t V,
                          int64_t E, uint64_t *keys, uint32_t *vals, BuildStatus *st) {
  int bad = 0, nself = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = col[i];
    const bool ok = v >= 0 && v < V;
    if (!ok || cap[i] < 0) bad++;
    if (ok && v == row_of[i]) nself++;
    keys[i] = ok ? (uint64_t)v : 0;
    vals[i] = (uint32_t)i;
  }
  bad = block_reduce_i32<false>(bad);
  nself = block_reduce_i32<false>(nself);
  if (threadIdx.x == 0) {
    if (bad) atomicAdd(&st->bad_input, bad);
    if (nself) atomicAdd(&st->nself, nself);
  }
}

// R[x] = arcs whose head is below x, x in [0, V]: first sorted head >= x.
__global__ void k_rc_inprefix(const uint64_t *keys, int64_t E, int32_t V, int32_t *R) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x <= V; x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = E;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (keys[mid] < (uint64_t)x) lo = mid + 1; else hi = mid;
    }
    R[x] = (int32_t)lo;
  }
}

// Forward entries (arc order: coalesced reads and writes).  A self-loop gets
// residual 0 both ways, so it never carries flow.
__global__ void k_rc_forward(const int32_t *row_of, const int32_t *col, const int32_t *cap, int64_t E, const int32_t *R,
                             int32_t vbase, int32_t mbase, int2 *ent, int32_t *cap0, int32_t *flow, int32_t *arc2ent) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = row_of[i], v = col[i];
    const int32_t c = u == v ? 0 : cap[i];
    const int32_t k = (int32_t)i + R[u];
    ent[k] = make_int2(vbase + v, c);
    cap0[k] = c;
    flow[k] = 0;
    arc2ent[i] = mbase + k;
  }
}

// Reverse entries (head order: sequential writes, gathered tails).
__global__ void k_rc_reverse(const int64_t *rp, const uint64_t *keys, const uint32_t *vals, const int32_t *row_of,
                             int64_t E, const int32_t *R, int32_t vbase, int32_t mbase, int2 *ent, int32_t *cap0,
                             int32_t *flow) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < E; j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = (int32_t)keys[j];
    const int32_t i = (int32_t)vals[j];
    const int32_t u = row_of[i];
    const int64_t r1 = rp[v + 1];
    if (r1 < 0 || r1 > E) continue;  // malformed row pointers: k_check_rowptr rejects the build
    const int32_t k = (int32_t)(r1 + j);
    ent[k] = make_int2((vbase + u) | RC_REV, mbase + i + R[u]);
    cap0[k] = 0;
    flow[k] = 0;  // unused: a reverse entry's flow lives at its forward entry
  }
}

__global__ void k_rc_rowb(const int64_t *rp, const int32_t *R, int32_t V, int64_t E, int32_t vbase, int32_t mbase,
                          int2 *rowb) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < V; x += (int64_t)gridDim.x * blockDim.x) {
    // clamped: a malformed build is rejected, but its rows must stay in range until then
    const int64_t lo = rp[x] < 0 ? 0 : (rp[x] > E ? E : rp[x]);
    const int64_t hi = rp[x + 1] < lo ? lo : (rp[x + 1] > E ? E : rp[x + 1]);
    rowb[vbase + x] = make_int2(mbase + (int32_t)(lo + R[x]), mbase + (int32_t)(hi + R[x + 1]));
  }
}

__global__ void k_rc_count(int64_t E, BuildStatus *st) {
  if (blockIdx.x == 0 && threadIdx.x == 0) st->M = (int32_t)(2 * E);
}

hipError_t build_residual_rcsr(const int64_t *row_ptr, const int32_t *col, const int32_t *cap, int32_t V, int64_t E,
                               const Arena &A, const Place &pl, void *scratch, BuildStatus *status_dev,
                               hipStream_t st) {
  Scratch s;
  carve_scratch(V, E, scratch, &s);
  hipError_t e = hipMemsetAsync(status_dev, 0, sizeof(BuildStatus), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(V + 1)), dim3(BT), 0, st, row_ptr, V, E, status_dev, s.rowcnt);
  if (E == 0) {
    e = excl_scan_i32(s.rowcnt, s.rptr, (int64_t)V + 1, nullptr, s.stemp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowb, dim3(grid_for(V)), dim3(BT), 0, st, s.rptr, V, pl.vbase, (int32_t)pl.mbase, A.rowb);
    return hipGetLastError();
  }
  const int vb = bits_for(V);
  // row of every arc (marks at the row starts and a prefix sum)
  e = hipMemsetAsync(s.head, 0, 4 * ((size_t)E + 1), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_row_marks, dim3(grid_for(V)), dim3(BT), 0, st, row_ptr, V, E, s.head);
  e = excl_scan_i32(s.head, s.hx, E + 1, nullptr, s.stemp, st);
  if (e != hipSuccess) return e;
  const int32_t *row_of = s.hx + 1;
  hipLaunchKernelGGL(k_rc_keys, dim3(grid_for(E)), dim3(BT), 0, st, row_ptr, row_of, col, cap, V, E, s.k0, s.v0,
                     status_dev);
  int alt = 0;
  e = radix_sort_u64_u32(s.k0, s.v0, s.k1, s.v1, E, vb, s.hist, s.stemp, &alt, st);
  if (e != hipSuccess) return e;
  const uint64_t *keys = alt ? s.k1 : s.k0;
  const uint32_t *vals = alt ? s.v1 : s.v0;
  int32_t *R = s.rptr;
  int32_t *flow = A.rev + pl.mbase;
  hipLaunchKernelGGL(k_rc_inprefix, dim3(grid_for((int64_t)V + 1)), dim3(BT), 0, st, keys, E, V, R);
  hipLaunchKernelGGL(k_rc_forward, dim3(grid_for(E)), dim3(BT), 0, st, row_of, col, cap, E, R, pl.vbase,
                     (int32_t)pl.mbase, A.ent + pl.mbase, A.cap0 + pl.mbase, flow, A.arc2ent + pl.abase);
  hipLaunchKernelGGL(k_rc_reverse, dim3(grid_for(E)), dim3(BT), 0, st, row_ptr, keys, vals, row_of, E, R, pl.vbase,
                     (int32_t)pl.mbase, A.ent + pl.mbase, A.cap0 + pl.mbase, flow);
  hipLaunchKernelGGL(k_rc_rowb, dim3(grid_for(V)), dim3(BT), 0, st, row_ptr, R, V, E, pl.vbase, (int32_t)pl.mbase,
                     A.rowb);
  hipLaunchKernelGGL(k_rc_count, dim3(1), dim3(1), 0, st, E, status_dev);
  return hipGetLastError();
}

hipError_t build_residual(const int64_t *row_ptr, const int32_t *col, const int32_t *cap, int32_t V, int64_t E,
                          const Arena &A, const Place &pl, void *scratch, BuildStatus *status_dev, hipStream_t st) {
  const int64_t N = 2 * E;
  Scratch s;
  carve_scratch(V, E, scratch, &s);
  int2 *ent = A.ent + pl.mbase;
  int32_t *rev = A.rev + pl.mbase;
  int32_t *cap0 = A.cap0 + pl.mbase;
  int32_t *arc2ent = A.arc2ent + pl.abase;
  int32_t *pbefore = A.pbefore + pl.abase;
  int32_t *acap = A.acap + pl.abase;
  hipError_t e = hipMemsetAsync(status_dev, 0, sizeof(BuildStatus), st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_check_rowptr, dim3(grid_for(V + 1)), dim3(BT), 0, st, row_ptr, V, E, status_dev, s.rowcnt);
  if (E == 0) {
    // no arcs: every row is empty
    e = excl_scan_i32(s.rowcnt, s.rptr, (int64_t)V + 1, nullptr, s.stemp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rowb, dim3(grid_for(V)), dim3(BT), 0, st, s.rptr, V, pl.vbase, (int32_t)pl.mbase, A.rowb);
    return hipGetLastError();
  }
  const int vb = bits_for(V);
  // The backward keys start where an odd number of radix passes on their
  // row bits leaves them in k0 + E, beside the forward keys in k0, so the
  // merge reads both from k0 and writes k1 with no copies in between.
  const bool odd = radix_sort_passes(vb) & 1;
  uint64_t *bk = odd ? s.k1 + E : s.k0 + E;
  uint32_t *bv = odd ? s.v1 + E : s.v0 + E;
  // keys, with each arc's row found in its tile's row starts (the tile
  // bounds' rows in hx, which is free until step 3)
  {
    const int64_t ntiles = (E + EK_TILE - 1) / EK_TILE;
    hipLaunchKernelGGL(k_tile_rows, dim3(grid_for(ntiles + 1)), dim3(BT), 0, st, row_ptr, V, E, ntiles, s.hx);
    const int64_t ngroups = (E + RADIX_TILE - 1) / RADIX_TILE;
    hipLaunchKernelGGL(k_emit_keys_tiled, dim3((unsigned)(ngroups < 65535 ? ngroups : 65535)), dim3(BT), 0, st,
                       row_ptr, s.hx, ntiles, col, cap, V, E, vb, s.k0, bk, bv, arc2ent, acap, s.hist, status_dev);
  }
  // which path: the host needs the row-order check (and the self-loop count)
  BuildStatus hs;
  e = hipMemcpyAsync(&hs, status_dev, sizeof(hs), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  const bool inline_self = hs.unsorted == 0;
  // the fused merge needs short runs of equal columns; a malformed input
  // (rejected after the build) takes the general steps
  const bool fused = inline_self && hs.longrun == 0 && hs.bad_input == 0;
  uint64_t *keys = nullptr;
  uint32_t *vals = nullptr;
  if (inline_self) {
    // backward keys: stable sort on their row bits only (emitted in arc
    // order, so equal rows stay ordered by the arc's tail), then merge with
    // the forward keys, which are sorted already
    int alt = 0;
    uint64_t *ok = odd ? s.k0 + E : s.k1 + E;
    uint32_t *ov = odd ? s.v0 + E : s.v1 + E;
    e = radix_sort_u64_u32(bk, bv, ok, ov, E, vb, s.hist, s.stemp, &alt, st, vb, true);
    if (e != hipSuccess) return e;
    if ((alt ? ok : bk) != s.k0 + E) {  // pass count disagrees with radix_sort_passes
      e = hipMemcpyAsync(s.k0 + E, alt ? ok : bk, 8 * (size_t)E, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(s.v0 + E, alt ? ov : bv, 4 * (size_t)E, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    if (fused) {
      // tile bounds, per-tile entry counts and their prefix sums in the
      // radix histogram's space (free after the sort; its 1,024 bytes per
      // 6,144 keys hold the 24 ntiles + 16 bytes); each entry's row in head[]
      const int64_t ntiles = (N + MT_TILE - 1) / MT_TILE;
      int64_t *split = (int64_t *)s.hist;
      int32_t *heads = (int32_t *)(split + 2 * (ntiles + 1));
      int32_t *hpre = heads + ntiles;
      const unsigned tgrid = (unsigned)(ntiles < 65535 ? ntiles : 65535);
      hipLaunchKernelGGL(k_merge_splits, dim3(grid_for(ntiles + 1)), dim3(BT), 0, st, s.k0, s.k0 + E, E, ntiles, split,
                         status_dev);
      hipLaunchKernelGGL(k_merge_count, dim3(tgrid), dim3(MT_THREADS), 0, st, s.k0, s.k0 + E, vb, ntiles, split, heads);
      e = excl_scan_i32(heads, hpre, ntiles, &status_dev->M, s.stemp, st);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_merge_entries, dim3(tgrid), dim3(MT_THREADS), 0, st, s.k0, s.k0 + E, s.v0 + E, E, vb, cap,
                         pl.vbase, ntiles, split, hpre, status_dev, ent, cap0, s.head, s.uid_of, pbefore);
      hipLaunchKernelGGL(k_rowptr_rows, dim3(grid_for((int64_t)V + 1)), dim3(BT), 0, st, s.head, V, status_dev,
                         s.rptr);
    } else {
      // the merge marks the group heads as it writes (row_of in hx is no
      // longer needed)
      hipLaunchKernelGGL(k_iota, dim3(grid_for(E)), dim3(BT), 0, st, s.v0, E);
      hipLaunchKernelGGL(k_merge, dim3(grid_for((N + MERGE_TILE - 1) / MERGE_TILE, 1)), dim3(MERGE_THREADS), 0, st,
                         s.k0, s.v0, s.k0 + E, s.v0 + E, E, s.k1, s.v1, s.head, vb);
      keys = s.k1;
      vals = s.v1;
    }
  } else {
    if (odd) {  // the full sort wants all keys contiguous in k0
      e = hipMemcpyAsync(s.k0 + E, bk, 8 * (size_t)E, hipMemcpyDeviceToDevice, st);
      if (e == hipSuccess) e = hipMemcpyAsync(s.v0 + E, bv, 4 * (size_t)E, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_iota, dim3(grid_for(E)), dim3(BT), 0, st, s.v0, E);
    if (hs.nself > 0) hipLaunchKernelGGL(k_selfloops_last, dim3(grid_for(N)), dim3(BT), 0, st, s.k0, N, vb);
    int alt = 0;
    e = radix_sort_u64_u32(s.k0, s.v0, s.k1, s.v1, N, 2 * vb, s.hist, s.stemp, &alt, st);
    if (e != hipSuccess) return e;
    keys = alt ? s.k1 : s.k0;
    vals = alt ? s.v1 : s.v0;
    hipLaunchKernelGGL(k_heads, dim3(grid_for(N)), dim3(BT), 0, st, keys, N, vb, inline_self, status_dev, s.head);
  }
  if (!fused) {
    e = excl_scan_i32(s.head, s.hx, N, &status_dev->M, s.stemp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_groups, dim3(grid_for(N)), dim3(BT), 0, st, keys, vals, N, vb, inline_self, cap, status_dev,
                       s.head, s.hx, pl.vbase, ent, cap0, s.uid_of, pbefore, s.gstart);
    hipLaunchKernelGGL(k_long_groups, dim3(256), dim3(BT), 0, st, keys, vals, N, vb, inline_self, cap, status_dev,
                       s.hx, pl.vbase, ent, cap0, s.uid_of, pbefore, s.gstart);
    hipLaunchKernelGGL(k_rowptr, dim3(grid_for((int64_t)V + 1)), dim3(BT), 0, st, keys, N, vb, inline_self, V,
                       status_dev, s.hx, s.rptr);
  }
  hipLaunchKernelGGL(k_rowb, dim3(grid_for(V)), dim3(BT), 0, st, s.rptr, V, pl.vbase, (int32_t)pl.mbase, A.rowb);
  hipLaunchKernelGGL(k_arcs, dim3(grid_for(E)), dim3(BT), 0, st, E, s.uid_of, (int32_t)pl.mbase, rev, arc2ent,
                     pbefore, status_dev);
  hipLaunchKernelGGL(k_pair_check, dim3(grid_for(N, 64 * BT)), dim3(BT), 0, st, rev, (int32_t)pl.mbase, ent,
                     status_dev);
  return hipGetLastError();
}

}  // namespace wb
