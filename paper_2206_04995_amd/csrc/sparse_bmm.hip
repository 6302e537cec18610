// SparseBMM (paper Sec. 2.4, Alg. 2): for every x row, the union of the
// sparse S rows S_sparse[y] over the y in R[x], without duplicates.  S_sparse
// in CSR is a collision-free hash table on y (row pointer = bucket header).
//
// The paper deduplicates with one z-vector (SPA) stamped with the current x
// so it never has to be cleared.  Here x rows run in parallel, so every
// wavefront owns a small LDS hash set sized to the row's work (cleared per
// row, cost proportional to the row), and rows whose work exceeds it use
// workgroups with an LDS bitmap over windows of the z range; in count mode
// the windows of one heavy row run as separate workgroups.
//
// Count mode writes the number of distinct z per row; write mode writes the
// sorted z ids of each row at off[x] - off[x_lo].
#include "common.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

constexpr int NT = 256;
constexpr int LIGHT_MAX = 1024;      // rows with at most this much work use a wave hash set
constexpr int HT_SLOTS = 2048;       // slots of one wave's hash set (load <= 1/2)
constexpr int SMALL_SLOTS = 512;     // the table of rows with w <= 256: more waves fit in LDS
constexpr int32_t EMPTY = 0x7FFFFFFF;
constexpr int HB_BITS = 1 << 19;     // heavy-row window: 64 KB of LDS
constexpr int HB_WORDS = HB_BITS / 32;

__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// per R CSR entry j: the sparse S row of its join key, as (start, length)
__global__ void k_entry_seg(const int32_t* __restrict__ rcol, const int32_t* __restrict__ spptr, int64_t j_lo,
                            int64_t j_hi, int32_t* __restrict__ seg0, int32_t* __restrict__ len) {
  for (int64_t j = j_lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < j_hi;
       j += int64_t(gridDim.x) * blockDim.x) {
    const int y = rcol[j];
    const int a = spptr[y];
    seg0[j] = a;
    len[j] = spptr[y + 1] - a;
  }
}

// w[x] = sum of the entry lengths of row x (difference of the entries' prefix sums)
__global__ void k_row_diff(const int32_t* __restrict__ rptr, const int64_t* __restrict__ E, int64_t j_lo, int64_t x_lo,
                           int64_t x_hi, int64_t* __restrict__ w) {
  for (int64_t x = x_lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < x_hi;
       x += int64_t(gridDim.x) * blockDim.x)
    w[x - x_lo] = E[rptr[x + 1] - j_lo] - E[rptr[x] - j_lo];
}

__device__ __forceinline__ uint32_t hash_slot(int32_t z, int log2t) {
  return (uint32_t(z) * 0x9E3779B1u) >> (32 - log2t);
}

// In-place ascending bitonic sort of t (power of two) LDS ints by one wave.
__device__ void wave_bitonic(int32_t* a, int t) {
  const int lane = lane_id();
  for (int k = 2; k <= t; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = lane; i < t; i += 64) {
        int ixj = i ^ j;
        if (ixj > i) {
          int32_t u = a[i], v = a[ixj];
          bool up = (i & k) == 0;
          if ((u > v) == up) {
            a[i] = v;
            a[ixj] = u;
          }
        }
      }
      lds_fence();
    }
  }
}

// Lanes hold segments [s0, s0 + len) of a z-sorted array; every entry lands
// on one lane (owner found by a search over the wave's prefix sums) and its
// bit is set in the LDS bitmap of window [wlo, wlo + HB_BITS).
__device__ __forceinline__ void wave_flat_scatter(int s0, int len, const int32_t* __restrict__ col, int32_t wlo,
                                                  uint32_t* bm) {
  const int lane = lane_id();
  const int incl = wave_scan_add_dpp(len);
  const int excl = incl - len;
  const int total = __shfl(incl, 63, 64);
  for (int t0 = 0; t0 < total; t0 += 64) {
    const int tt = t0 + lane;
    int o = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int e = __shfl(excl, o + step, 64);
      if (e <= tt) o += step;
    }
    const int os0 = __shfl(s0, o, 64);
    const int oex = __shfl(excl, o, 64);
    if (tt < total) {
      const int d = col[os0 + (tt - oex)] - wlo;
      atomicOr(&bm[d >> 5], 1u << (d & 31));
    }
  }
}

// every thread takes join keys of the row, finds the part of its sparse S row
// inside the window by binary search, and its wave scatters the entries
__device__ __forceinline__ void heavy_window(const int32_t* __restrict__ seg0, const int32_t* __restrict__ seglen,
                                             const int32_t* __restrict__ spcol, int a, int b, int32_t wlo,
                                             int32_t whi, uint32_t* bm) {
  for (int c0 = a; c0 < b; c0 += NT) {
    const int j = c0 + int(threadIdx.x);
    int lo = 0, len = 0;
    if (j < b) {
      const int s0 = seg0[j], s1 = s0 + seglen[j];
      if (s1 > s0) {
        lo = int(lower_bound_dev<int32_t>(spcol, s0, s1, wlo));
        len = int(lower_bound_dev<int32_t>(spcol, lo, s1, whi)) - lo;
      }
    }
    wave_flat_scatter(lo, len, spcol, wlo, bm);
  }
}

// Rows with w in (W_LO, SLOTS / 2] (a table of SLOTS slots stays at most half
// full).  The launch with W_LO = 0 also writes the zero counts of empty and
// heavy rows (count mode), so every row's count is set before the heavy
// kernels add to it.
template <bool WRITE, int SLOTS, int W_LO>
__global__ void __launch_bounds__(NT) k_sparse_light(const int32_t* __restrict__ rptr, const int32_t* __restrict__ seg0,
                                                     const int32_t* __restrict__ seglen,
                                                     const int32_t* __restrict__ spcol, int64_t x_lo, int64_t x_hi,
                                                     const int64_t* __restrict__ w, int32_t* __restrict__ cnt,
                                                     const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ int32_t tab_all[NT / 64][SLOTS];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  int32_t* tab = tab_all[wid];
  const int64_t gw = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  const int64_t base_off = WRITE ? off[x_lo] : 0;

  for (int64_t x = x_lo + gw; x < x_hi; x += nw) {
    const int64_t wx = w[x - x_lo];
    if (wx > LIGHT_MAX || wx == 0) {
      // heavy rows are counted by the windowed kernel, which adds to cnt[x]
      if (!WRITE && W_LO == 0 && lane == 0) cnt[x] = 0;
      continue;
    }
    if (wx <= W_LO || wx > SLOTS / 2) continue;  // the other table size's rows
    int log2t = 6;
    while ((1 << log2t) < 2 * wx) ++log2t;
    const int t = 1 << log2t;
    for (int i = lane; i < t; i += 64) tab[i] = EMPTY;
    lds_fence();
    int fresh = 0;
    const int a = rptr[x], b = rptr[x + 1];
    for (int c0 = a; c0 < b; c0 += 64) {
      int j = c0 + lane;
      int s0 = 0, len = 0;
      if (j < b) {
        s0 = seg0[j];
        len = seglen[j];
      }
      int incl = wave_scan_add_dpp(len);
      int excl = incl - len;
      int total = __shfl(incl, 63, 64);
      for (int t0 = 0; t0 < total; t0 += 64) {
        int tt = t0 + lane;
        int o = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
          int e = __shfl(excl, o + step, 64);
          if (e <= tt) o += step;
        }
        int os0 = __shfl(s0, o, 64);
        int oex = __shfl(excl, o, 64);
        if (tt < total) {
          int32_t z = spcol[os0 + (tt - oex)];
          uint32_t h = hash_slot(z, log2t);
          while (true) {
            int32_t old = atomicCAS(&tab[h], EMPTY, z);
            if (old == EMPTY) {
              ++fresh;
              break;
            }
            if (old == z) break;
            h = (h + 1) & uint32_t(t - 1);
          }
        }
      }
    }
    int count = wave_sum(fresh);
    if (!WRITE) {
      if (lane == 0) cnt[x] = count;
    } else {
      lds_fence();
      wave_bitonic(tab, t);
      int32_t* dst = out + (off[x] - base_off);
      for (int i = lane; i < count; i += 64) dst[i] = tab[i];
    }
    lds_fence();
  }
}

// list of the heavy rows (order irrelevant: every row owns its output range)
__global__ void k_collect_heavy(int64_t x_lo, int64_t x_hi, const int64_t* __restrict__ w, int32_t* __restrict__ list,
                                int32_t* __restrict__ n_list) {
  for (int64_t x = x_lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < x_hi;
       x += int64_t(gridDim.x) * blockDim.x)
    if (w[x - x_lo] > LIGHT_MAX) list[atomicAdd(n_list, 1)] = int32_t(x);
}

// count mode: one workgroup per (heavy row, window blockIdx.y)
__global__ void __launch_bounds__(NT) k_sparse_heavy_count(const int32_t* __restrict__ rptr,
                                                           const int32_t* __restrict__ seg0,
                                                           const int32_t* __restrict__ seglen,
                                                           const int32_t* __restrict__ spcol, int n_inst,
                                                           const int32_t* __restrict__ x_base,
                                                           const int32_t* __restrict__ z_base,
                                                           const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ n_list,
                                                           int32_t* __restrict__ cnt) {
  __shared__ uint32_t bm[HB_WORDS];
  __shared__ int red[NT / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int nh = *n_list;
  for (int i = blockIdx.x; i < nh; i += gridDim.x) {
    const int64_t x = list[i];
    const int inst = n_inst == 1 ? 0 : find_inst<int32_t>(x_base, n_inst, int32_t(x));
    const int32_t zlo = z_base[inst], zhi = z_base[inst + 1];
    const int64_t wlo64 = int64_t(zlo) + int64_t(blockIdx.y) * HB_BITS;
    if (wlo64 >= zhi) continue;
    const int32_t wlo = int32_t(wlo64);
    const int32_t whi = (zhi - wlo) > HB_BITS ? wlo + HB_BITS : zhi;
    for (int i = threadIdx.x; i < HB_WORDS; i += NT) bm[i] = 0u;
    __syncthreads();
    heavy_window(seg0, seglen, spcol, rptr[x], rptr[x + 1], wlo, whi, bm);
    __syncthreads();
    constexpr int PER = HB_WORDS / NT;
    int c = 0;
    for (int k = 0; k < PER; ++k) c += __popc(bm[threadIdx.x * PER + k]);
    c = wave_sum(c);
    if (lane == 0) red[wid] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int q = 0; q < NT / 64; ++q) tot += red[q];
      if (tot) atomicAdd(&cnt[x], tot);
    }
    __syncthreads();
  }
}

// write mode: one workgroup per heavy row, windows in z order
__global__ void __launch_bounds__(NT) k_sparse_heavy_write(const int32_t* __restrict__ rptr,
                                                           const int32_t* __restrict__ seg0,
                                                           const int32_t* __restrict__ seglen,
                                                           const int32_t* __restrict__ spcol, int n_inst,
                                                           const int32_t* __restrict__ x_base,
                                                           const int32_t* __restrict__ z_base, int64_t x_lo,
                                                           const int32_t* __restrict__ list,
                                                           const int32_t* __restrict__ n_list,
                                                           const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ uint32_t bm[HB_WORDS];
  __shared__ int red[NT / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t base_off = off[x_lo];
  const int nh = *n_list;

  for (int i = blockIdx.x; i < nh; i += gridDim.x) {
    const int64_t x = list[i];
    const int inst = n_inst == 1 ? 0 : find_inst<int32_t>(x_base, n_inst, int32_t(x));
    const int32_t zlo = z_base[inst], zhi = z_base[inst + 1];
    int64_t wpos = off[x] - base_off;
    for (int64_t wlo64 = zlo; wlo64 < zhi; wlo64 += HB_BITS) {
      const int32_t wlo = int32_t(wlo64);
      const int32_t whi = (zhi - wlo) > HB_BITS ? wlo + HB_BITS : zhi;
      for (int i = threadIdx.x; i < HB_WORDS; i += NT) bm[i] = 0u;
      __syncthreads();
      heavy_window(seg0, seglen, spcol, rptr[x], rptr[x + 1], wlo, whi, bm);
      __syncthreads();
      // thread t owns words [t*PER, (t+1)*PER): contiguous, so prefix order is z order
      constexpr int PER = HB_WORDS / NT;
      int c = 0;
      for (int k = 0; k < PER; ++k) c += __popc(bm[threadIdx.x * PER + k]);
      int inc = wave_incl_scan(c);
      if (lane == 63) red[wid] = inc;
      __syncthreads();
      int pre = 0, tot = 0;
      for (int q = 0; q < NT / 64; ++q) {
        int v = red[q];
        if (q < wid) pre += v;
        tot += v;
      }
      int64_t pos = wpos + pre + (inc - c);
      for (int k = 0; k < PER; ++k) {
        uint32_t word = bm[threadIdx.x * PER + k];
        while (word) {
          int bit = __ffs(word) - 1;
          word &= word - 1;
          out[pos++] = wlo + (threadIdx.x * PER + k) * 32 + bit;
        }
      }
      wpos += tot;
      __syncthreads();
    }
  }
}

}  // namespace

void sparse_row_work(const RowCtx& c, int64_t x_lo, int64_t x_hi, int64_t j_lo, int64_t j_hi, int64_t* w,
                     int32_t* seg0, int32_t* seglen, hipStream_t s, Arena& a) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  const int64_t ne = j_hi - j_lo;
  int64_t* E = a.alloc<int64_t>(ne + 1, s);
  if (ne > 0) {
    int g = int(std::min<int64_t>((ne + NT - 1) / NT, 1 << 16));
    hipLaunchKernelGGL(k_entry_seg, dim3(g), dim3(NT), 0, s, c.rcol, c.spptr, j_lo, j_hi, seg0, seglen);
    JP_LAUNCH_CHECK();
  }
  scan_excl_i32_to_i64(seglen + j_lo, E, ne, s, a);
  int g = int(std::min<int64_t>((n + NT - 1) / NT, 1 << 16));
  hipLaunchKernelGGL(k_row_diff, dim3(g), dim3(NT), 0, s, c.rptr, E, j_lo, x_lo, x_hi, w);
  JP_LAUNCH_CHECK();
  a.give_back(E, s);
}

void sparse_bmm(const RowCtx& c, int64_t x_lo, int64_t x_hi, const int64_t* w, int32_t* cnt, const int64_t* off,
                int32_t* out, int32_t* heavy_list, hipStream_t s) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  int gl = int(std::min<int64_t>((n + 3) / 4, 1 << 15));
  int gh = int(std::min<int64_t>(n, 1024));
  // heavy_list holds n + 1 ints: the count, then the rows
  int32_t* n_list = heavy_list;
  int32_t* list = heavy_list + 1;
  fill_i32(n_list, 1, 0, s);
  hipLaunchKernelGGL(k_collect_heavy, dim3(int(std::min<int64_t>((n + NT - 1) / NT, 4096))), dim3(NT), 0, s, x_lo, x_hi,
                     w, list, n_list);
  JP_LAUNCH_CHECK();
  if (out) {
    hipLaunchKernelGGL((k_sparse_light<true, SMALL_SLOTS, 0>), dim3(gl), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen,
                       c.spcol, x_lo, x_hi, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sparse_light<true, HT_SLOTS, SMALL_SLOTS / 2>), dim3(gl), dim3(NT), 0, s, c.rptr, c.seg0,
                       c.seglen, c.spcol, x_lo, x_hi, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sparse_heavy_write, dim3(gh), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen, c.spcol, c.n_inst,
                       c.x_base, c.z_base, x_lo, list, n_list, off, out);
    JP_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL((k_sparse_light<false, SMALL_SLOTS, 0>), dim3(gl), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen,
                       c.spcol, x_lo, x_hi, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sparse_light<false, HT_SLOTS, SMALL_SLOTS / 2>), dim3(gl), dim3(NT), 0, s, c.rptr, c.seg0,
                       c.seglen, c.spcol, x_lo, x_hi, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    const int wins = int(std::max<int64_t>(1, (c.max_z_range + HB_BITS - 1) / HB_BITS));
    hipLaunchKernelGGL(k_sparse_heavy_count, dim3(gh, wins), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen, c.spcol,
                       c.n_inst, c.x_base, c.z_base, list, n_list, cnt);
    JP_LAUNCH_CHECK();
  }
}

}  // namespace jp
