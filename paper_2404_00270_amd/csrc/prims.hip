// Device-wide primitives for the residual-graph builder: exclusive prefix sum
// and a stable least-significant-digit radix sort of 64-bit keys carrying a
// 32-bit payload.  Written for wave64: ranks inside a wave come from ballots,
// ranks across the waves of a workgroup from LDS counters.
#include "wb_common.h"
#include "wb_internal.h"

namespace wb {

// ------------------------------------------------------------------ scan
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
#pragma unroll
  for (int d = 1; d < WB_WAVE; d <<= 1) {
    T y;
    if constexpr (sizeof(T) == 8) {
      unsigned lo = (unsigned)((unsigned long long)x), hi = (unsigned)((unsigned long long)x >> 32);
      lo = (unsigned)__shfl_up((int)lo, d, WB_WAVE);
      hi = (unsigned)__shfl_up((int)hi, d, WB_WAVE);
      y = (T)(((unsigned long long)hi << 32) | lo);
    } else {
      y = (T)__shfl_up((int)x, d, WB_WAVE);
    }
    if (lane() >= d) x += y;
  }
  return x;
}

// Exclusive scan of a workgroup's per-thread values; returns the thread's
// exclusive prefix and writes the workgroup total to *total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *total) {
  __shared__ T wsum[SCAN_THREADS / WB_WAVE];
  T incl = wave_incl_scan(x);
  int w = threadIdx.x / WB_WAVE;
  if (lane() == WB_WAVE - 1) wsum[w] = incl;
  __syncthreads();
  T off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < SCAN_THREADS / WB_WAVE; i++) {
    T v = wsum[i];
    if (i < w) off += v;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return off + incl - x;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const TI *in, int64_t n, TO *partial) {
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  TO acc = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    int64_t i = base + (int64_t)j * SCAN_THREADS + threadIdx.x;
    if (i < n) acc += (TO)in[i];
  }
  TO tot;
  block_excl_scan<TO>(acc, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of the per-tile totals in place; writes
// the grand total to *total_out.
template <typename TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_partials(TO *partial, int64_t nb, TO *total_out) {
  TO carry = 0;
  for (int64_t base = 0; base < nb; base += SCAN_THREADS) {
    int64_t i = base + threadIdx.x;
    TO v = i < nb ? partial[i] : (TO)0;
    TO tot;
    TO ex = block_excl_scan<TO>(v, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename TI, typename TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_down(const TI *in, TO *out, int64_t n, const TO *partial) {
  __shared__ TO tile[SCAN_TILE];
  int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    int idx = j * SCAN_THREADS + threadIdx.x;
    int64_t i = base + idx;
    tile[idx] = i < n ? (TO)in[i] : (TO)0;
  }
  __syncthreads();
  TO loc[SCAN_ITEMS];
  TO acc = 0;
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    loc[j] = acc;
    acc += tile[threadIdx.x * SCAN_ITEMS + j];
  }
  TO tot;
  TO off = block_excl_scan<TO>(acc, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) tile[threadIdx.x * SCAN_ITEMS + j] = loc[j] + off;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < SCAN_ITEMS; j++) {
    int idx = j * SCAN_THREADS + threadIdx.x;
    int64_t i = base + idx;
    if (i < n) out[i] = tile[idx];
  }
}

int64_t scan_temp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

template <typename TI, typename TO>
static hipError_t scan_impl(const TI *in, TO *out, int64_t n, TO *total, TO *temp, hipStream_t st) {
  int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nb == 0) {
    if (total) return hipMemsetAsync(total, 0, sizeof(TO), st);
    return hipSuccess;
  }
  hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, n, temp);
  hipLaunchKernelGGL((k_scan_partials<TO>), dim3(1), dim3(SCAN_THREADS), 0, st, temp, nb, total);
  hipLaunchKernelGGL((k_scan_down<TI, TO>), dim3((unsigned)nb), dim3(SCAN_THREADS), 0, st, in, out, n, temp);
  return hipGetLastError();
}

hipError_t excl_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *total, int32_t *temp, hipStream_t st) {
  return scan_impl<int32_t, int32_t>(in, out, n, total, temp, st);
}

// ------------------------------------------------------------- radix sort
constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / WB_WAVE;
constexpr int RS_ITEMS = 24;  // 6,144 keys a tile: 78 KB of LDS in the scatter, two workgroups a CU
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
static_assert(RS_THREADS == RS_BINS, "one thread per digit in the scatter's set-up");
static_assert(RS_TILE == RADIX_TILE && RS_BITS == RADIX_BITS, "tile and digit that producers of a first histogram use");

// hist[d * nblocks + b] = number of items of tile b whose digit is d.
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t *keys, int64_t n, int shift, int32_t *hist,
                                                       int nblocks) {
  __shared__ int cnt[RS_BINS];
  for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) cnt[d] = 0;
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * RS_TILE;
  // every key of the thread is loaded before the first count, so all its
  // loads are in flight together
  uint64_t kk[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; j++) {
    const int64_t i = base + (int64_t)j * RS_THREADS + threadIdx.x;
    kk[j] = i < n ? keys[i] : 0;
  }
#pragma unroll
  for (int j = 0; j < RS_ITEMS; j++) {
    const int64_t i = base + (int64_t)j * RS_THREADS + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(kk[j] >> shift) & (RS_BINS - 1)], 1);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < RS_BINS; d += RS_THREADS) hist[(int64_t)d * nblocks + blockIdx.x] = cnt[d];
}

// Stable scatter through LDS.  Wave w of the workgroup owns items
// [w * RS_ITEMS * 64, (w + 1) * RS_ITEMS * 64) of the tile, read 64 at a
// time (coalesced).  Phase 1 ranks every item among the earlier items of its
// wave with the same digit, against wave-private digit counters in LDS (no
// workgroup barrier between rounds: a wave's LDS accesses stay in order).
// Then the counters become per-wave offsets within each digit, the tile is
// placed in LDS in (digit, index) order, and written out so that
// consecutive threads store consecutive positions of one digit's run.
// Stable: within a digit, items keep (wave, round, lane) = index order.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t *kin, const uint32_t *vin, uint64_t *kout,
                                                          uint32_t *vout, int64_t n, int shift,
                                                          const int32_t *hist_scanned, int nblocks) {
  __shared__ uint64_t s_key[RS_TILE];
  __shared__ uint32_t s_val[RS_TILE];
  __shared__ int s_gbase[RS_BINS];  // global position of this tile's first item of digit d
  __shared__ int s_lbase[RS_BINS];  // LDS position of this tile's first item of digit d
  __shared__ int s_wcnt[RS_WAVES][RS_BINS];
  __shared__ int s_wsum[RS_WAVES];
  const int w = threadIdx.x / WB_WAVE;
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const int tile_n = (int)(n - base < RS_TILE ? n - base : RS_TILE);
  {
    const int d = threadIdx.x;  // RS_THREADS == RS_BINS
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ww++) s_wcnt[ww][d] = 0;
  }
  __syncthreads();
  // phase 1: rank within the wave's range
  volatile int *wc = s_wcnt[w];
  const unsigned long long lt = lanemask_lt();
  const int wbase = w * RS_ITEMS * WB_WAVE;
  uint64_t kk[RS_ITEMS];
  uint32_t vv[RS_ITEMS];
  int rr[RS_ITEMS];
#pragma unroll
  for (int j = 0; j < RS_ITEMS; j++) {
    const int li = wbase + j * WB_WAVE + lane();
    const bool valid = li < tile_n;
    kk[j] = valid ? kin[base + li] : 0;
    vv[j] = valid ? vin[base + li] : 0;
  }
#pragma unroll
  for (int j = 0; j < RS_ITEMS; j++) {
    const int li = wbase + j * WB_WAVE + lane();
    const bool valid = li < tile_n;
    const int d = (int)((kk[j] >> shift) & (RS_BINS - 1));
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; b++) {
      const unsigned long long bits = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bits : ~bits;
    }
    const int rank = __popcll(peers & lt);
    __builtin_amdgcn_wave_barrier();
    const int before = valid ? wc[d] : 0;
    __builtin_amdgcn_wave_barrier();
    rr[j] = before + rank;
    if (valid && rank == 0) wc[d] = before + __popcll(peers);
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // per digit: offsets of the waves, tile total, digit bases
  {
    const int d = threadIdx.x;
    int acc = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ww++) {
      const int c = s_wcnt[ww][d];
      s_wcnt[ww][d] = acc;
      acc += c;
    }
    const int64_t idx = (int64_t)d * nblocks + blockIdx.x;
    s_gbase[d] = hist_scanned[idx];
    int incl = acc;
#pragma unroll
    for (int o = 1; o < WB_WAVE; o <<= 1) {
      const int y = __shfl_up(incl, o, WB_WAVE);
      if (lane() >= o) incl += y;
    }
    if (lane() == WB_WAVE - 1) s_wsum[w] = incl;
    __syncthreads();
    int off = 0;
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ww++) off += ww < w ? s_wsum[ww] : 0;
    s_lbase[d] = off + incl - acc;
  }
  __syncthreads();
  // phase 2: place the tile in LDS in (digit, index) order
#pragma unroll
  for (int j = 0; j < RS_ITEMS; j++) {
    const int li = wbase + j * WB_WAVE + lane();
    if (li < tile_n) {
      const int d = (int)((kk[j] >> shift) & (RS_BINS - 1));
      const int pos = s_lbase[d] + s_wcnt[w][d] + rr[j];
      s_key[pos] = kk[j];
      s_val[pos] = vv[j];
    }
  }
  __syncthreads();
  // write out: position p of digit d goes to gbase[d] + p - lbase[d]
  for (int p = threadIdx.x; p < tile_n; p += RS_THREADS) {
    const uint64_t key = s_key[p];
    const int d = (int)((key >> shift) & (RS_BINS - 1));
    const int64_t gp = (int64_t)s_gbase[d] + (p - s_lbase[d]);
    kout[gp] = key;
    vout[gp] = s_val[p];
  }
}

int64_t radix_hist_elems(int64_t n) { return (int64_t)RS_BINS * ((n + RS_TILE - 1) / RS_TILE); }

// Sorts (k0,v0) stably on key bits [shift0, shift0 + bits); (k1,v1) is
// scratch of the same size.  *result_in_alt is set when the sorted data ends
// in (k1,v1).
int radix_sort_passes(int bits) { return (bits + RS_BITS - 1) / RS_BITS; }

hipError_t radix_sort_u64_u32(uint64_t *k0, uint32_t *v0, uint64_t *k1, uint32_t *v1, int64_t n, int bits,
                              int32_t *hist, int32_t *scan_temp, int *result_in_alt, hipStream_t st, int shift0,
                              bool first_hist) {
  *result_in_alt = 0;
  if (n <= 1) return hipSuccess;
  int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
  int64_t hn = (int64_t)RS_BINS * nblocks;
  uint64_t *ka = k0, *kb = k1;
  uint32_t *va = v0, *vb = v1;
  for (int shift = shift0; shift < shift0 + bits; shift += RS_BITS) {
    if (!(first_hist && shift == shift0))
      hipLaunchKernelGGL(k_rs_hist, dim3(nblocks), dim3(RS_THREADS), 0, st, ka, n, shift, hist, nblocks);
    hipError_t e = excl_scan_i32(hist, hist, hn, nullptr, scan_temp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblocks), dim3(RS_THREADS), 0, st, ka, va, kb, vb, n, shift, hist, nblocks);
    uint64_t *tk = ka; ka = kb; kb = tk;
    uint32_t *tv = va; va = vb; vb = tv;
    *result_in_alt ^= 1;
  }
  return hipGetLastError();
}

}  // namespace wb
