// Shared device helpers for the HIP max-flow path (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define WB_WAVE 64

// Excess of a terminal carries this bias so that e > 0 never holds for it:
// the active test e(u) > 0 && h(u) < hcap then excludes s and t with no
// vertex-id comparison.  |bias| exceeds any reachable sum of int32
// capacities over < 2^31 arcs.
#define WB_EXCESS_BIAS (-(1LL << 62))

#define WB_KEY_NONE (~0ull)

namespace wb {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

__device__ __forceinline__ unsigned long long lanemask_lt() {
  return (1ull << lane()) - 1ull;
}

// 64-bit xor shuffle built from two 32-bit lane permutes.
__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long v, int m) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = (unsigned)__shfl_xor((int)lo, m, WB_WAVE);
  hi = (unsigned)__shfl_xor((int)hi, m, WB_WAVE);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long v, int src) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = (unsigned)__shfl((int)lo, src, WB_WAVE);
  hi = (unsigned)__shfl((int)hi, src, WB_WAVE);
  return ((unsigned long long)hi << 32) | lo;
}

// Minimum over aligned groups of P lanes (P a power of two <= 64).  Every
// lane of the wave must execute this (converged control flow).
__device__ __forceinline__ unsigned long long shfl_up_u64(unsigned long long v, int d) {
  unsigned lo = (unsigned)v, hi = (unsigned)(v >> 32);
  lo = (unsigned)__shfl_up((int)lo, d, WB_WAVE);
  hi = (unsigned)__shfl_up((int)hi, d, WB_WAVE);
  return ((unsigned long long)hi << 32) | lo;
}

template <int P>
__device__ __forceinline__ unsigned long long group_min(unsigned long long k) {
#pragma unroll
  for (int m = P >> 1; m > 0; m >>= 1) {
    unsigned long long o = shfl_xor_u64(k, m);
    k = o < k ? o : k;
  }
  return k;
}

template <int P>
__device__ __forceinline__ long long group_sum_i64(long long x) {
#pragma unroll
  for (int m = P >> 1; m > 0; m >>= 1) x += (long long)shfl_xor_u64((unsigned long long)x, m);
  return x;
}

__device__ __forceinline__ int wave_sum_i32(int x) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += __shfl_xor(x, m, WB_WAVE);
  return x;
}

// Relaxed device-scope atomics (coherent across the XCDs' L2 caches).
__device__ __forceinline__ long long atomic_load_i64(const long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_load_i32(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_load_u64(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long atomic_add_i64(long long *p, long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_add_i32(int *p, int v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_add_u64(unsigned long long *p, unsigned long long v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_min_u64(unsigned long long *p, unsigned long long v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int atomic_or_i32(int *p, int v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long atomic_cas_i64(long long *p, long long expected, long long desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value found (== the expected one on success)
}
__device__ __forceinline__ void atomic_store_i32(int *p, int v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-aggregated append: lanes with pred set write val into q at
// consecutive slots reserved by one atomic on *cnt.  Slots at or beyond
// `cap` are not written; they bump *err instead (a queue can only overflow
// through a bug, which the host then reports).  Lanes that do not take part
// may be inactive; the active ones need not be converged beyond that.
__device__ __forceinline__ void wave_append(bool pred, int val, int *q, int *cnt, int cap, int *err) {
  unsigned long long m = __ballot(pred);
  if (m == 0) return;
  int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane() == leader) base = atomic_add_i32(cnt, __popcll(m));
  base = __shfl(base, leader, WB_WAVE);
  if (pred) {
    int idx = base + __popcll(m & lanemask_lt());
    if (idx < cap) q[idx] = val;
    else atomic_add_i32(err, 1);
  }
}

// Per-wave LDS staging for queue appends: a wave collects up to WB_QBUF
// entries in its own LDS slice and moves them to the global queue with one
// atomic on the global counter, instead of one atomic per append.  Lanes of
// a wave run in lockstep, so the wave-private LDS counter needs no barrier;
// divergent sub-groups of a wave execute one after the other.
#define WB_QBUF 512

struct WaveQ {
  int *buf;  // LDS staging slice of this wave (lcap entries)
  int *cnt;  // LDS counter for this wave
  int *gq;   // global queue
  int *gcnt; // global counter
  int gcap;  // global capacity
  int *err;  // overflow counter
  int lcap = WB_QBUF;
};

__device__ __forceinline__ void waveq_flush(const WaveQ &q) {
  __builtin_amdgcn_wave_barrier();
  const int c = *(volatile int *)q.cnt;
  if (c == 0) return;
  const unsigned long long act = __ballot(true);
  const int leader = __ffsll((long long)act) - 1;
  const int na = __popcll(act);
  const int r = __popcll(act & lanemask_lt());
  int base = 0;
  if (lane() == leader) base = atomic_add_i32(q.gcnt, c);
  base = __shfl(base, leader, WB_WAVE);
  for (int j = r; j < c; j += na) {
    const int idx = base + j;
    const int v = ((volatile int *)q.buf)[j];
    if (idx < q.gcap) q.gq[idx] = v;
    else atomic_add_i32(q.err, 1);
  }
  __builtin_amdgcn_wave_barrier();
  if (lane() == leader) *(volatile int *)q.cnt = 0;
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ void waveq_push(const WaveQ &q, bool pred, int val) {
  const unsigned long long m = __ballot(pred);
  if (m == 0) return;
  const int n = __popcll(m);
  __builtin_amdgcn_wave_barrier();
  int c = *(volatile int *)q.cnt;
  if (c + n > q.lcap) {
    waveq_flush(q);
    c = 0;
  }
  if (pred) ((volatile int *)q.buf)[c + __popcll(m & lanemask_lt())] = val;
  __builtin_amdgcn_wave_barrier();
  if (lane() == __ffsll((long long)m) - 1) *(volatile int *)q.cnt = c + n;
  __builtin_amdgcn_wave_barrier();
}

// Final flush of the WaveQ of every wave of a workgroup (WAVES waves), with
// one atomic on the global counter for the whole workgroup: atomics on one
// address serialise, and one per wave costs thousands per launch.  Every
// thread of the workgroup calls it, converged; s_off is LDS scratch of
// WAVES + 1 ints, free again when it returns.
template <int WAVES>
__device__ __forceinline__ void block_flush(const WaveQ &q, int *s_off) {
  const int w = threadIdx.x / WB_WAVE;
  __builtin_amdgcn_wave_barrier();
  const int c = *(volatile int *)q.cnt;
  if (lane() == 0) s_off[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int i = 0; i < WAVES; i++) {
      const int x = s_off[i];
      s_off[i] = tot;
      tot += x;
    }
    s_off[WAVES] = tot ? atomic_add_i32(q.gcnt, tot) : 0;
  }
  __syncthreads();
  const int base = s_off[WAVES] + s_off[w];
  for (int j = lane(); j < c; j += WB_WAVE) {
    const int idx = base + j;
    const int v = ((volatile int *)q.buf)[j];
    if (idx < q.gcap) q.gq[idx] = v;
    else atomic_add_i32(q.err, 1);
  }
  __builtin_amdgcn_wave_barrier();
  if (lane() == 0) *(volatile int *)q.cnt = 0;
  __syncthreads();  // s_off may be reused at once
}

// Grid-wide barrier for cooperative launches (all workgroups co-resident).
// Two levels: workgroups count on the cache line of their group
// (blockIdx % WB_BAR_GROUPS, which follows the round-robin placement of
// workgroups on the 8 XCDs), the last of each group counts at the root, and
// the last group bumps the generation everyone polls.  Measured on MI355X
// with 256 workgroups: about 7 us per barrier, against 20 us for a single
// shared counter (66 us at 1024 workgroups).  Release/acquire fences at
// device scope make prior global writes visible across the XCDs' L2s.
// Layout of bar[]: [0] generation, [16] root count, [32 + 16 g] group g.
#define WB_BAR_GROUPS 8
#define WB_BAR_WORDS (32 + 16 * WB_BAR_GROUPS)

__device__ __forceinline__ void grid_barrier(unsigned *bar, unsigned nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned *gen = &bar[0];
    unsigned *root = &bar[16];
    const unsigned g = blockIdx.x % WB_BAR_GROUPS;
    unsigned *grp = &bar[32 + 16 * g];
    const unsigned gsize = nblocks / WB_BAR_GROUPS + (g < nblocks % WB_BAR_GROUPS ? 1u : 0u);
    const unsigned ngroups = nblocks < WB_BAR_GROUPS ? nblocks : WB_BAR_GROUPS;
    const unsigned gv = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this block's writes
    bool last = false;
    if (__hip_atomic_fetch_add(grp, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gsize - 1) {
      __hip_atomic_store(grp, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__hip_atomic_fetch_add(root, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ngroups - 1) {
        __hip_atomic_store(root, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gv) __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

}  // namespace wb
