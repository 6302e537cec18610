// The classical Join-Project solution (paper Sec. 1.1) on the device, and the
// strategy choice f1 between it and the hybrid DIM^3 path (Sec. 2.6).
//
// Classical path: a hash join with S as the build side (open-addressing table
// on S.y holding each key's count; S.z grouped by key behind it), then
// deduplication of the projected join rows (x, z) in a device hash set of
// 64-bit keys.  No mapping, no partition.  The count is the number of keys
// that enter the set; the sorted list comes from compacting the set and two
// stable radix sorts (z, then x).
//
// f1 (Sec. 2.6) compares the mapping cost the classical path avoids,
// 2 (|R| + |S|) t_map, with the deduplication cost it pays beyond SparseBMM's,
// |OUT_J| (t_hash - t_randRW): the classical path is taken when
// OUT_J < ratio * (|R| + |S|).  OUT_J is estimated from a sample of R.y and
// S.y (exact when both sides have at most SAMPLE tuples).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "classical.h"
#include "common.h"
#include "prim.h"

namespace jp {
namespace {

constexpr int NT = 256;
constexpr int SAMPLE = 4096;  // tuples per side in the OUT_J estimate
constexpr int SAMPLE_NT = 1024;
constexpr int64_t EMPTY_Y = INT64_MIN;         // free slot of the S.y table
constexpr uint64_t EMPTY_K = ~uint64_t(0);     // free slot of a 64-bit key set
constexpr uint32_t EMPTY_V = 0xFFFFFFFFu;      // free slot of a 32-bit value set

inline int grid(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 1 << 20))); }

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

__device__ __forceinline__ uint64_t pair_key(int32_t x, int32_t z) {
  return (uint64_t(uint32_t(x) ^ 0x80000000u) << 32) | uint64_t(uint32_t(z) ^ 0x80000000u);
}
__device__ __forceinline__ uint64_t slot_of_y(int32_t y, int shift) {
  return (uint64_t(uint32_t(y)) * 0x9E3779B97F4A7C15ull) >> shift;
}

// ---------------------------------------------------------------- f1 estimate

// matches = number of (sampled R tuple, sampled S tuple) pairs with equal y;
// the samples take every sr-th (ss-th) tuple, mr (ms) of them.  The S sample
// goes into an LDS hash table of key counts (load <= 1/2), the R sample probes it.
constexpr int SLOTS = 2 * SAMPLE;
__global__ void __launch_bounds__(SAMPLE_NT) k_sample_matches(const int32_t* __restrict__ ry, int64_t sr, int mr,
                                                              const int32_t* __restrict__ sy, int64_t ss, int ms,
                                                              unsigned long long* __restrict__ matches) {
  __shared__ int32_t key[SLOTS];
  __shared__ int32_t cnt[SLOTS];
  __shared__ int32_t min_cnt;  // the key INT32_MIN is the free marker: counted apart
  __shared__ unsigned long long tot;
  for (int i = threadIdx.x; i < SLOTS; i += SAMPLE_NT) {
    key[i] = INT32_MIN;
    cnt[i] = 0;
  }
  if (threadIdx.x == 0) {
    min_cnt = 0;
    tot = 0;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ms; i += SAMPLE_NT) {
    const int32_t y = sy[int64_t(i) * ss];
    if (y == INT32_MIN) {
      atomicAdd(&min_cnt, 1);
      continue;
    }
    uint32_t h = (uint32_t(y) * 0x9E3779B1u) >> (32 - 13);
    while (true) {
      const int32_t old = atomicCAS(&key[h], INT32_MIN, y);
      if (old == INT32_MIN || old == y) break;
      h = (h + 1) & (SLOTS - 1);
    }
    atomicAdd(&cnt[h], 1);
  }
  __syncthreads();
  unsigned long long mine = 0;
  for (int i = threadIdx.x; i < mr; i += SAMPLE_NT) {
    const int32_t y = ry[int64_t(i) * sr];
    if (y == INT32_MIN) {
      mine += (unsigned long long)min_cnt;
      continue;
    }
    uint32_t h = (uint32_t(y) * 0x9E3779B1u) >> (32 - 13);
    while (true) {
      const int32_t k = key[h];
      if (k == y) {
        mine += (unsigned long long)cnt[h];
        break;
      }
      if (k == INT32_MIN) break;
      h = (h + 1) & (SLOTS - 1);
    }
  }
  atomicAdd(&tot, mine);
  __syncthreads();
  if (threadIdx.x == 0) *matches = tot;
}

// ---------------------------------------------------------------- hash join

// S.y into the open-addressing table: slot per tuple, count per key
__global__ void k_build_s(const int32_t* __restrict__ sy, int64_t n, int64_t* __restrict__ key,
                          int32_t* __restrict__ cnt, int shift, uint64_t mask, int64_t* __restrict__ slot_out) {
  GRID_STRIDE(i, n) {
    const int32_t y = sy[i];
    uint64_t s = slot_of_y(y, shift);
    while (true) {
      int64_t k = key[s];
      if (k == EMPTY_Y) {
        k = int64_t(atomicCAS(reinterpret_cast<unsigned long long*>(&key[s]), (unsigned long long)EMPTY_Y,
                              (unsigned long long)int64_t(y)));
        if (k == EMPTY_Y) k = y;
      }
      if (k == int64_t(y)) break;
      s = (s + 1) & mask;
    }
    atomicAdd(&cnt[s], 1);
    slot_out[i] = int64_t(s);
  }
}

// S.z grouped by the slot of its y: zlist[cur[slot]++] = z
__global__ void k_group_s(const int32_t* __restrict__ sz, const int64_t* __restrict__ slot, int64_t n,
                          int32_t* __restrict__ cur, int32_t* __restrict__ zlist) {
  GRID_STRIDE(i, n) { zlist[atomicAdd(&cur[slot[i]], 1)] = sz[i]; }
}

// probe: the slot of each R tuple's y (-1 if y is not in S) and its number of S partners
__global__ void k_probe_r(const int32_t* __restrict__ ry, int64_t n, const int64_t* __restrict__ key,
                          const int32_t* __restrict__ cnt, int shift, uint64_t mask, int64_t* __restrict__ rslot,
                          int32_t* __restrict__ deg) {
  GRID_STRIDE(i, n) {
    const int32_t y = ry[i];
    uint64_t s = slot_of_y(y, shift);
    int64_t found = -1;
    while (true) {
      const int64_t k = key[s];
      if (k == int64_t(y)) {
        found = int64_t(s);
        break;
      }
      if (k == EMPTY_Y) break;
      s = (s + 1) & mask;
    }
    rslot[i] = found;
    deg[i] = found >= 0 ? cnt[found] : 0;
  }
}

// distinct values of a column (optionally only entries whose rslot >= 0) in a
// 32-bit set whose free marker is EMPTY_V; the value EMPTY_V itself sets *extra
// instead; *count receives every value that entered either
__global__ void k_distinct(const int32_t* __restrict__ v, const int64_t* __restrict__ keep, int64_t n,
                           uint32_t* __restrict__ set, int shift, uint64_t mask, int32_t* __restrict__ extra,
                           unsigned long long* __restrict__ count) {
  GRID_STRIDE(i, n) {
    bool fresh = false;
    if (!keep || keep[i] >= 0) {
      const uint32_t u = uint32_t(v[i]);
      if (u == EMPTY_V) {
        fresh = atomicExch(extra, 1) == 0;
      } else {
        uint64_t s = (uint64_t(u) * 0x9E3779B97F4A7C15ull) >> shift;
        while (true) {
          uint32_t k = set[s];
          if (k == EMPTY_V) {
            k = atomicCAS(&set[s], EMPTY_V, u);
            if (k == EMPTY_V) {
              fresh = true;
              break;
            }
          }
          if (k == u) break;
          s = (s + 1) & mask;
        }
      }
    }
    const uint64_t m = ballot(fresh);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(count, (unsigned long long)__popcll(m));
  }
}

// deduplication: every join row (R tuple i, its j-th S partner) puts
// key(x, z) into the set; keys that enter it are counted
__global__ void k_dedup(const int32_t* __restrict__ rx, const int64_t* __restrict__ rslot,
                        const int64_t* __restrict__ jr_off, int n_r, int64_t out_j,
                        const int32_t* __restrict__ start, const int32_t* __restrict__ zlist,
                        uint64_t* __restrict__ set, int shift, uint64_t mask, int32_t* __restrict__ extra,
                        unsigned long long* __restrict__ count) {
  SegCursor<int64_t> cur(jr_off, n_r);
  cur.seed(chunk_first() < out_j ? chunk_first() : 0);
  CHUNK_LOOP(j, out_j, JP_CHUNK) {
    const int i = cur(j);
    const int32_t z = zlist[start[rslot[i]] + (j - cur.lo)];
    const uint64_t k = pair_key(rx[i], z);
    bool fresh = false;
    if (k == EMPTY_K) {
      fresh = atomicExch(extra, 1) == 0;
    } else {
      uint64_t s = mix64(k) >> shift;
      while (true) {
        unsigned long long o = set[s];
        if (o == EMPTY_K) {
          o = atomicCAS(reinterpret_cast<unsigned long long*>(&set[s]), (unsigned long long)EMPTY_K,
                        (unsigned long long)k);
          if (o == EMPTY_K) {
            fresh = true;
            break;
          }
        }
        if (o == k) break;
        s = (s + 1) & mask;
      }
    }
    const uint64_t m = ballot(fresh);
    if (m && lane_id() == __ffsll((unsigned long long)m) - 1) atomicAdd(count, (unsigned long long)__popcll(m));
  }
}

__global__ void k_positive(const int32_t* __restrict__ v, int64_t n, int32_t* __restrict__ f) {
  GRID_STRIDE(i, n) { f[i] = v[i] > 0 ? 1 : 0; }
}

__global__ void k_occupied(const uint64_t* __restrict__ set, int64_t cap, int32_t* __restrict__ flag) {
  GRID_STRIDE(i, cap) { flag[i] = set[i] != EMPTY_K ? 1 : 0; }
}

// set entries as (z word, x word) of their keys, compacted; the key of
// (INT32_MAX, INT32_MAX) (the free marker) goes last when present
__global__ void k_compact_keys(const uint64_t* __restrict__ set, int64_t cap, const int32_t* __restrict__ flag,
                               const int32_t* __restrict__ E, const int32_t* __restrict__ extra,
                               uint32_t* __restrict__ kz, uint32_t* __restrict__ kx) {
  GRID_STRIDE(i, cap) {
    if (flag[i]) {
      const uint64_t k = set[i];
      kz[E[i]] = uint32_t(k);
      kx[E[i]] = uint32_t(k >> 32);
    }
    if (i == cap - 1 && *extra) {
      kz[E[cap]] = 0xFFFFFFFFu;
      kx[E[cap]] = 0xFFFFFFFFu;
    }
  }
}

__global__ void k_unflip(const uint32_t* __restrict__ kx, const uint32_t* __restrict__ kz, int64_t n,
                         int32_t* __restrict__ ox, int32_t* __restrict__ oz) {
  GRID_STRIDE(i, n) {
    ox[i] = int32_t(kx[i] ^ 0x80000000u);
    oz[i] = int32_t(kz[i] ^ 0x80000000u);
  }
}

// rows of the sorted result: heads of runs of equal x
__global__ void k_x_heads(const int32_t* __restrict__ x, int64_t n, int32_t* __restrict__ flag) {
  GRID_STRIDE(i, n) { flag[i] = (i == 0 || x[i] != x[i - 1]) ? 1 : 0; }
}

__global__ void k_x_rows(const int32_t* __restrict__ x, const int32_t* __restrict__ flag,
                         const int32_t* __restrict__ E, int64_t n, int32_t* __restrict__ xv,
                         int64_t* __restrict__ off) {
  GRID_STRIDE(i, n) {
    if (flag[i]) {
      xv[E[i]] = x[i];
      off[E[i]] = i;
    }
    if (i == n - 1) off[E[n]] = n;
  }
}

void lc() { JP_LAUNCH_CHECK(); }

int log2_ceil(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

void d2h_sync(void* dst, const void* src, size_t bytes, hipStream_t s) {
  JP_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));
}

}  // namespace

void launch_out_j_sample(const int32_t* ry, int64_t nr, const int32_t* sy, int64_t ns, unsigned long long* matches,
                         hipStream_t s) {
  if (nr == 0 || ns == 0) {
    fill_i64(reinterpret_cast<int64_t*>(matches), 1, 0, s);
    return;
  }
  const int64_t sr = (nr + SAMPLE - 1) / SAMPLE, ss = (ns + SAMPLE - 1) / SAMPLE;
  const int mr = int((nr + sr - 1) / sr), ms = int((ns + ss - 1) / ss);
  hipLaunchKernelGGL(k_sample_matches, dim3(1), dim3(SAMPLE_NT), 0, s, ry, sr, mr, sy, ss, ms, matches);
  lc();
}

int64_t out_j_from_sample(unsigned long long matches, int64_t nr, int64_t ns) {
  if (nr == 0 || ns == 0) return 0;
  const int64_t sr = (nr + SAMPLE - 1) / SAMPLE, ss = (ns + SAMPLE - 1) / SAMPLE;
  const int mr = int((nr + sr - 1) / sr), ms = int((ns + ss - 1) / ss);
  return int64_t(std::llround(double(matches) * (double(nr) / mr) * (double(ns) / ms)));
}

int64_t estimate_out_j(const int32_t* ry, int64_t nr, const int32_t* sy, int64_t ns, hipStream_t s) {
  Arena T;
  unsigned long long* d = T.alloc<unsigned long long>(1, s);
  launch_out_j_sample(ry, nr, sy, ns, d, s);
  unsigned long long m = 0;
  d2h_sync(&m, d, sizeof(m), s);
  T.release(s);
  return out_j_from_sample(m, nr, ns);
}

bool f1_prefers_classical(int64_t out_j_est, int64_t nr, int64_t ns) {
  const char* v = std::getenv("JP_F1_RATIO");
  const double ratio = v ? std::atof(v) : JP_F1_RATIO_DEFAULT;
  return double(out_j_est) < ratio * double(nr + ns);
}

void ClassicalPlan::build(const int32_t* rx_, const int32_t* ry, int64_t nr_, const int32_t* sz, const int32_t* sy,
                          int64_t ns_, bool timing, hipStream_t s) {
  stream = s;
  rx = rx_;
  nr = nr_;
  ns = ns_;
  if (timing) {
    for (auto& e : ev) JP_HIP(hipEventCreate(&e));
    JP_HIP(hipEventRecord(ev[0], s));
  }
  Arena T(&B);
  // build side: S.y table (load <= 1/2)
  shift_s = 64 - std::max(1, log2_ceil(std::max<int64_t>(2 * ns, 2)));
  cap_s = int64_t(1) << (64 - shift_s);
  skey = A.alloc<int64_t>(cap_s, s);
  fill_i64(skey, cap_s, EMPTY_Y, s);
  int32_t* cnt = T.alloc<int32_t>(cap_s, s);
  fill_i32(cnt, cap_s, 0, s);
  int64_t* sslot = T.alloc<int64_t>(std::max<int64_t>(ns, 1), s);
  if (ns) hipLaunchKernelGGL(k_build_s, dim3(grid(ns)), dim3(NT), 0, s, sy, ns, skey, cnt, shift_s,
                             uint64_t(cap_s - 1), sslot);
  lc();
  start = A.alloc<int32_t>(cap_s + 1, s);
  scan_excl_i32(cnt, start, cap_s, s, T);
  int32_t* cur = T.alloc<int32_t>(cap_s, s);
  JP_HIP(hipMemcpyAsync(cur, start, cap_s * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  zlist = A.alloc<int32_t>(std::max<int64_t>(ns, 1), s);
  if (ns) hipLaunchKernelGGL(k_group_s, dim3(grid(ns)), dim3(NT), 0, s, sz, sslot, ns, cur, zlist);
  lc();
  // probe side: partners per R tuple, OUT_J
  rslot = A.alloc<int64_t>(std::max<int64_t>(nr, 1), s);
  int32_t* deg = T.alloc<int32_t>(std::max<int64_t>(nr, 1), s);
  if (nr) hipLaunchKernelGGL(k_probe_r, dim3(grid(nr)), dim3(NT), 0, s, ry, nr, skey, cnt, shift_s,
                             uint64_t(cap_s - 1), rslot, deg);
  lc();
  jr_off = A.alloc<int64_t>(nr + 1, s);
  scan_excl_i32_to_i64(deg, jr_off, nr, s, T);
  // statistics: distinct y of S (occupied slots), kept R tuples, distinct x of them, distinct z of S
  unsigned long long* dc = T.alloc<unsigned long long>(4, s);
  int32_t* extra = T.alloc<int32_t>(4, s);
  fill_i64(reinterpret_cast<int64_t*>(dc), 4, 0, s);
  fill_i32(extra, 4, 0, s);
  auto distinct = [&](const int32_t* v, const int64_t* keep, int64_t n, int k) {
    if (n == 0) return;
    const int sh = 64 - std::max(1, log2_ceil(std::max<int64_t>(2 * n, 2)));
    const int64_t cap = int64_t(1) << (64 - sh);
    uint32_t* set = T.alloc<uint32_t>(cap, s);
    fill_u32(set, cap, EMPTY_V, s);
    hipLaunchKernelGGL(k_distinct, dim3(grid(n)), dim3(NT), 0, s, v, keep, n, set, sh, uint64_t(cap - 1),
                       extra + k, dc + k);
    lc();
    T.give_back(set, s);
  };
  distinct(sy, nullptr, ns, 0);
  distinct(rx, rslot, nr, 1);
  distinct(sz, nullptr, ns, 2);
  int64_t* d_kept = T.alloc<int64_t>(1, s);
  fill_i64(d_kept, 1, 0, s);
  if (nr) {
    // kept R tuples: those with at least one partner
    int32_t* kept = T.alloc<int32_t>(nr, s);
    hipLaunchKernelGGL(k_positive, dim3(grid(nr)), dim3(NT), 0, s, deg, nr, kept);
    lc();
    reduce_sum_i32_to_i64(kept, nr, d_kept, s);
  }
  unsigned long long h[4];
  int64_t hk = 0;
  JP_HIP(hipMemcpyAsync(h, dc, sizeof(h), hipMemcpyDeviceToHost, s));
  JP_HIP(hipMemcpyAsync(&hk, d_kept, sizeof(hk), hipMemcpyDeviceToHost, s));
  JP_HIP(hipMemcpyAsync(&out_j, jr_off + nr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));
  n_y = int64_t(h[0]);  // the extra flags are counted by the kernels already
  n_x = int64_t(h[1]);
  n_z = int64_t(h[2]);
  n_r_kept = hk;
  T.release(s);
  if (timing) JP_HIP(hipEventRecord(ev[1], s));
}

void ClassicalPlan::execute(hipStream_t s) {
  if (timing_on()) JP_HIP(hipEventRecord(ev[2], s));
  if (!set) {
    shift_d = 64 - std::max(10, log2_ceil(std::max<int64_t>(2 * out_j, 2)));
    cap_d = int64_t(1) << (64 - shift_d);
    set = A.alloc<uint64_t>(cap_d, s);
    d_cnt = A.alloc<unsigned long long>(1, s);
    d_extra = A.alloc<int32_t>(1, s);
  }
  fill_i64(reinterpret_cast<int64_t*>(set), cap_d, int64_t(EMPTY_K), s);
  fill_i64(reinterpret_cast<int64_t*>(d_cnt), 1, 0, s);
  fill_i32(d_extra, 1, 0, s);
  if (out_j > 0)
    hipLaunchKernelGGL(k_dedup, dim3(chunk_grid(out_j)), dim3(NT), 0, s, rx, rslot, jr_off, int(nr), out_j, start,
                       zlist, set, shift_d, uint64_t(cap_d - 1), d_extra, d_cnt);
  lc();
  if (timing_on()) JP_HIP(hipEventRecord(ev[3], s));
  executed = true;
  have_total = false;
  sorted = false;
}

void ClassicalPlan::fetch_total(hipStream_t s) {
  if (!executed) throw Error(JP_ESTATE, "count before execute");
  if (have_total) return;
  unsigned long long c = 0;  // keys that entered the set, the flagged key included
  JP_HIP(hipMemcpyAsync(&c, d_cnt, sizeof(c), hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));
  total = int64_t(c);
  have_total = true;
}

void ClassicalPlan::sort_result(hipStream_t s) {
  fetch_total(s);
  if (sorted) return;
  Arena T(&B);
  const int64_t n = total;
  int32_t* flag = T.alloc<int32_t>(cap_d, s);
  hipLaunchKernelGGL(k_occupied, dim3(grid(cap_d)), dim3(NT), 0, s, set, cap_d, flag);
  lc();
  int32_t* E = T.alloc<int32_t>(cap_d + 1, s);
  scan_excl_i32(flag, E, cap_d, s, T);
  uint32_t* kz = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
  uint32_t* kx = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
  uint32_t* kz2 = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
  uint32_t* kx2 = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
  hipLaunchKernelGGL(k_compact_keys, dim3(grid(cap_d)), dim3(NT), 0, s, set, cap_d, flag, E, d_extra, kz, kx);
  lc();
  // LSD: z word, then x word (stable), on all 32 bits of each
  if (radix_sort_pairs(kz, kx, kz2, kx2, n, 32, s, T)) {
    std::swap(kz, kz2);
    std::swap(kx, kx2);
  }
  if (radix_sort_pairs(kx, kz, kx2, kz2, n, 32, s, T)) {
    std::swap(kx, kx2);
    std::swap(kz, kz2);
  }
  sx = A.alloc<int32_t>(std::max<int64_t>(n, 1), s);
  sz_ = A.alloc<int32_t>(std::max<int64_t>(n, 1), s);
  if (n) hipLaunchKernelGGL(k_unflip, dim3(grid(n)), dim3(NT), 0, s, kx, kz, n, sx, sz_);
  lc();
  // rows: distinct x (n_x of them: every kept R tuple yields a pair) and their offsets
  xv = A.alloc<int32_t>(std::max<int64_t>(n_x, 1), s);
  xoff = A.alloc<int64_t>(n_x + 1, s);
  if (n) {
    int32_t* hf = T.alloc<int32_t>(n, s);
    int32_t* HE = T.alloc<int32_t>(n + 1, s);
    hipLaunchKernelGGL(k_x_heads, dim3(grid(n)), dim3(NT), 0, s, sx, n, hf);
    lc();
    scan_excl_i32(hf, HE, n, s, T);
    hipLaunchKernelGGL(k_x_rows, dim3(grid(n)), dim3(NT), 0, s, sx, hf, HE, n, xv, xoff);
    lc();
  } else {
    fill_i64(xoff, 1, 0, s);
  }
  JP_HIP(hipStreamSynchronize(s));
  T.release(s);
  sorted = true;
}

int64_t ClassicalPlan::materialize(int part, int64_t first, int64_t maxp, int32_t* ox, int32_t* oz, hipStream_t s) {
  fetch_total(s);
  const int64_t count = part == JP_PART_DENSE ? 0 : total;
  if (first > count) throw Error(JP_ERANGE, "first beyond the number of pairs");
  const int64_t nw = std::min(maxp, count - first);
  if (nw <= 0) return 0;
  sort_result(s);
  JP_HIP(hipMemcpyAsync(ox, sx + first, nw * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  JP_HIP(hipMemcpyAsync(oz, sz_ + first, nw * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  JP_HIP(hipStreamSynchronize(s));
  return nw;
}

void ClassicalPlan::row_info(int part, int32_t* x_values, int64_t* row_offsets, hipStream_t s) {
  if (!executed) {
    if (row_offsets) throw Error(JP_ESTATE, "row offsets before execute");
    if (x_values && n_x > 0) throw Error(JP_ESTATE, "the classical path lists its x values after execute");
    return;
  }
  sort_result(s);
  if (x_values && n_x) JP_HIP(hipMemcpyAsync(x_values, xv, n_x * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  if (row_offsets) {
    if (part == JP_PART_DENSE) {
      std::fill(row_offsets, row_offsets + n_x + 1, int64_t(0));
    } else {
      JP_HIP(hipMemcpyAsync(row_offsets, xoff, (n_x + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    }
  }
  JP_HIP(hipStreamSynchronize(s));
}

void ClassicalPlan::stats(jp_stats* st) const {
  std::memset(st, 0, sizeof(*st));
  st->n_x = n_x;
  st->n_y = n_y;
  st->n_z = n_z;
  st->n_r_kept = n_r_kept;
  st->out_j = out_j;
  st->tau = INT64_MAX;
  st->footprint_bytes = A.bytes();
  st->peak_bytes = B.peak;
  st->strategy = JP_STRATEGY_CLASSICAL;
}

void ClassicalPlan::timings(jp_timings* t, hipStream_t s) {
  if (!executed || !ev[0]) throw Error(JP_ESTATE, "timings need JP_FLAG_TIMING and a jp_execute");
  JP_HIP(hipStreamSynchronize(s));
  std::memset(t, 0, sizeof(*t));
  JP_HIP(hipEventElapsedTime(&t->map_ms, ev[0], ev[1]));
  JP_HIP(hipEventElapsedTime(&t->sparse_ms, ev[2], ev[3]));
  t->execute_ms = t->sparse_ms;
}

ClassicalPlan::~ClassicalPlan() {
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  A.release(stream);
}

}  // namespace jp
