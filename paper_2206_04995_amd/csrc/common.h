// Internal helpers shared by the HIP sources of the Join-Project library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define JP_WAVE 64

namespace jp {

// ---------------------------------------------------------------- device

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

// Inclusive prefix maximum over the 64 lanes in DPP, with the shifts and row
// broadcasts of wave_scan_add_dpp (a maximum may see a lane twice).  Lanes a
// DPP step does not write take INT32_MIN.  Needs all 64 lanes active.
__device__ __forceinline__ int wave_scan_max_dpp(int x) {
  const int lo = INT32_MIN;
  int v = max(x, __builtin_amdgcn_update_dpp(lo, x, 0x111, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, x, 0x112, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, x, 0x113, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xF, 0xE, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x118, 0xF, 0xC, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x142, 0xA, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x143, 0xC, 0xF, false));
  return v;
}

// Sum over the 64 lanes without LDS traffic: DPP permutations reduce each
// 16-lane row (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror), then the four row sums are read as scalars.  Wave-uniform result.
__device__ __forceinline__ int wave_sum_dpp(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true);
  v += __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true);
  return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) + __builtin_amdgcn_readlane(v, 32) +
         __builtin_amdgcn_readlane(v, 48);
}

// Inclusive prefix sum over the 64 lanes in DPP, without LDS: three row shifts
// of the input give sums of 4 inside each 16-lane row, shifts by 4 and 8 (on
// the upper banks) complete the rows, and the row broadcasts of lanes 15 and 31
// carry row totals into the rows above.  Lanes a DPP step does not write take
// 0.  Needs all 64 lanes active.
__device__ __forceinline__ int wave_scan_add_dpp(int x) {
  int v = x + __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, x, 0x113, 0xF, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xE, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xC, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
  return v;
}

// inclusive prefix sum across the 64 lanes of a wave
template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (l >= o) v += u;
  }
  return v;
}

// index of the instance owning element g: base[] has n_inst + 1 ascending entries
template <class T>
__device__ __forceinline__ int find_inst(const T* __restrict__ base, int n_inst, T g) {
  int lo = 0, hi = n_inst;  // answer in [0, n_inst)
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (base[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

// find_inst by the whole wave (all 64 lanes, uniform control flow): a 64-ary
// search with one load per lane and level (two levels up to 4096 segments)
// instead of a chain of dependent loads.  Wave-uniform result.
template <class T>
__device__ __forceinline__ int wave_find_inst(const T* __restrict__ base, int n_inst, T g) {
  if (n_inst <= 1) return 0;
  const int lane = lane_id();
  int lo = 0, span = n_inst;  // the answer is in [lo, lo + span)
  while (span > 1) {
    const int step = (span + 63) >> 6;
    const int idx = lo + lane * step;
    const uint64_t m = __ballot(idx < lo + span && base[idx] <= g);
    if (m == 0) break;  // g below base[0]
    const int k = 63 - __builtin_clzll((unsigned long long)m);
    const int nlo = lo + k * step;
    span = min(step, lo + span - nlo);
    lo = nlo;
  }
  return lo;
}

// Segment index of increasing positions: the first call searches, later calls
// step forward (or search again after a long gap).  Loops over contiguous
// chunks (CHUNK_LOOP) keep the steps short, so most lookups cost one load.
template <class T>
struct SegCursor {
  const T* base;
  int n;
  int cur = -1;
  T lo = 0, hi = 0;  // base[cur], base[cur + 1]: a query inside costs no load
  __device__ SegCursor(const T* b, int n_) : base(b), n(n_) {}
  __device__ void set(int c) {
    cur = c;
    lo = base[c];
    hi = base[c + 1];
  }
  // Wave-cooperative start (all 64 lanes, uniform control flow) at the
  // segment of g0; g0 should not exceed the wave's later queries (a wrong
  // seed costs a search later, not a wrong answer).
  __device__ void seed(T g0) {
    if (n <= 1) {
      if (n == 1) set(0);
      else cur = 0;
      return;
    }
    set(wave_find_inst<T>(base, n, g0));
  }
  __device__ int operator()(T g) {
    if (n == 1) {
      if (cur < 0) set(0);
      return 0;
    }
    if (cur >= 0 && g >= lo && g < hi) return cur;
    if (cur < 0 || g < lo) {
      set(find_inst<T>(base, n, g));
      return cur;
    }
    int c = cur;
    for (int steps = 0; g >= base[c + 1]; ++steps) {
      if (steps == 8) {
        set(find_inst<T>(base, n, g));
        return cur;
      }
      ++c;
    }
    set(c);
    return cur;
  }
};

// Block b covers elements [b * ch, (b + 1) * ch) of [0, n); its threads stride
// by blockDim inside the chunk, so each thread's positions grow in small steps.
#define CHUNK_LOOP(i, n, ch)                                                                     \
  for (int64_t i = int64_t(blockIdx.x) * (ch) + threadIdx.x,                                      \
               i##_end = (int64_t(blockIdx.x) + 1) * (ch) < int64_t(n) ? (int64_t(blockIdx.x) + 1) * (ch) \
                                                                   : int64_t(n);                   \
       i < i##_end; i += blockDim.x)

constexpr int JP_CHUNK = 4096;  // elements per block of CHUNK_LOOP kernels (256 threads x 16)

// first element of this block's CHUNK_LOOP chunk
__device__ __forceinline__ int64_t chunk_first() { return int64_t(blockIdx.x) * JP_CHUNK; }

inline int chunk_grid(int64_t n, int ch = JP_CHUNK) { return int(n <= 0 ? 1 : (n + ch - 1) / ch); }

// first index in [lo, hi) with a[i] >= v (a ascending)
template <class T>
__device__ __forceinline__ int64_t lower_bound_dev(const T* __restrict__ a, int64_t lo, int64_t hi, T v) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < v) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  // SplitMix64 output finaliser (Steele, Lea, Flood 2014; constants of splitmix64)
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }


// ------------------------------------------------- decoupled look-back
// Single-pass prefix over tiles (Merrill and Garland, "Single-pass Parallel
// Prefix Scan with Decoupled Look-back", 2016).  A tile takes its index from a
// counter (status[ntiles]) in the order tiles start, publishes its own total,
// sums what its predecessors published until it meets an inclusive prefix,
// and publishes its own inclusive prefix.  A status word holds a flag in its
// top two bits (1: tile total, 2: inclusive prefix, 0: not yet published) and
// the value as a 62-bit two's complement integer, so one 64-bit store
// publishes both.  status[0, ntiles + 2) starts at zero.  A tile only waits on
// tiles that took their index before it, which are running or done, so every
// wait ends; the wait is bounded all the same (status[ntiles + 1] records a
// wait that gave up).
constexpr uint64_t LB_VALUE_MASK = (uint64_t(1) << 62) - 1;
constexpr int LB_SPIN_MAX = 1 << 16;

__device__ __forceinline__ uint64_t lb_pack(uint64_t flag, int64_t v) {
  return (flag << 62) | (uint64_t(v) & LB_VALUE_MASK);
}
__device__ __forceinline__ int64_t lb_value(uint64_t w) { return int64_t(w << 2) >> 2; }

// thread 0 of the block: the tile index, in start order
__device__ __forceinline__ int64_t lookback_ticket(uint64_t* status, int64_t ntiles) {
  return int64_t(atomicAdd(reinterpret_cast<unsigned long long*>(status + ntiles), 1ull));
}

// one whole wave: returns the sum of the totals of tiles [0, tile) and
// publishes this tile's inclusive prefix
__device__ __forceinline__ int64_t lookback_exclusive(uint64_t* status, int64_t tile, int64_t ntiles, int64_t total) {
  const int lane = lane_id();
  int64_t excl = 0;
  if (tile == 0) {
    if (lane == 0) __hip_atomic_store(status, lb_pack(2, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0) __hip_atomic_store(status + tile, lb_pack(1, total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  // lane l reads tile t - l; the window moves back 64 tiles until it holds an inclusive prefix
  for (int64_t t = tile - 1;; t -= 64) {
    const int64_t idx = t - lane;
    uint64_t w;
    for (int spin = 0;; ++spin) {
      w = idx >= 0 ? __hip_atomic_load(status + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : lb_pack(2, 0);
      if (ballot((w >> 62) == 0) == 0) break;
      if (spin == LB_SPIN_MAX) {
        if (lane == 0) atomicOr(reinterpret_cast<unsigned long long*>(status + ntiles + 1), 1ull);
        w = lb_pack(2, 0);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    const uint64_t incm = ballot((w >> 62) == 2);
    const int stop = incm ? __ffsll((unsigned long long)incm) - 1 : 63;
    excl += wave_sum(lane <= stop ? lb_value(w) : int64_t(0));
    if (incm) break;
  }
  if (lane == 0)
    __hip_atomic_store(status + tile, lb_pack(2, excl + total), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

}  // namespace jp
