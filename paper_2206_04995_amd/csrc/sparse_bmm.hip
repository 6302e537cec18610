// SparseBMM (paper Sec. 2.4, Alg. 2): for every x row, the union of the
// sparse S rows S_sparse[y] over the y in R[x], without duplicates.  S_sparse
// in CSR is a collision-free hash table on y (row pointer = bucket header).
//
// The paper deduplicates with one z-vector (SPA) stamped with the current x
// so it never has to be cleared.  Here x rows run in parallel, each with its
// own LDS set, chosen by the row's work w (join rows reaching sparse z): rows
// are first sorted into lists by w, then light rows (w <= 1024) run one per
// wavefront with a hash set sized to the row (cleared per row, cost
// proportional to the row), medium rows (count mode, w <= 8192) one per
// workgroup with a shared hash set, and heavy rows as workgroups with an LDS
// bitmap over windows of the z range (in count mode the windows of one row run
// as separate workgroups).
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
constexpr int MED_MAX = 8192;       // count mode: rows up to this much work use a workgroup hash set
constexpr int HB_BITS = 1 << 19;     // heavy-row window: 64 KB of LDS
constexpr int HB_WORDS = HB_BITS / 32;

__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// per R CSR entry j: the sparse S row of its join key, as (start, length)
__global__ void k_entry_seg(const int32_t* __restrict__ rcol, const int32_t* __restrict__ spptr, int64_t j_lo,
                            int64_t j_hi, int32_t* __restrict__ seg0, int32_t* __restrict__ len) {
  // a block per chunk of JP_CHUNK entries, eight entries per thread and step:
  // their column loads, then their row-pointer gathers, then the stores
  constexpr int U = 8;
  const int64_t c0 = j_lo + int64_t(blockIdx.x) * JP_CHUNK;
  const int64_t c1 = c0 + JP_CHUNK < j_hi ? c0 + JP_CHUNK : j_hi;
  const int64_t step = blockDim.x;
  for (int64_t j0 = c0 + threadIdx.x; j0 < c1; j0 += U * step) {
    int32_t y[U], a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) y[u] = rcol[j0 + u * step < c1 ? j0 + u * step : c1 - 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = spptr[y[u]];
      b[u] = spptr[y[u] + 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * step;
      if (j < c1) {
        seg0[j] = a[u];
        len[j] = b[u] - a[u];
      }
    }
  }
}

// w[x] = sum of the entry lengths of row x: one thread per row (rows are a
// few entries long on average and their lengths lie together); a row of more
// than ROW_LONG entries goes to a list that whole workgroups sum
constexpr int ROW_LONG = 512;

__global__ void k_row_work(const int32_t* __restrict__ rptr, const int32_t* __restrict__ len, int64_t x_lo,
                           int64_t x_hi, int64_t* __restrict__ w, int32_t* __restrict__ long_rows,
                           int32_t* __restrict__ n_long) {
  for (int64_t x = x_lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x; x < x_hi;
       x += int64_t(gridDim.x) * blockDim.x) {
    const int32_t a = rptr[x], b = rptr[x + 1];
    if (b - a > ROW_LONG) {
      long_rows[atomicAdd(n_long, 1)] = int32_t(x);
      continue;
    }
    // four lengths' loads in flight per step
    int64_t sum = 0;
    int32_t j = a;
    for (; j + 4 <= b; j += 4) {
      const int32_t l0 = len[j], l1 = len[j + 1], l2 = len[j + 2], l3 = len[j + 3];
      sum += int64_t(l0) + l1 + l2 + l3;
    }
    for (; j < b; ++j) sum += len[j];
    w[x - x_lo] = sum;
  }
}

__global__ void __launch_bounds__(NT) k_row_work_long(const int32_t* __restrict__ rptr, const int32_t* __restrict__ len,
                                                      int64_t x_lo, int64_t* __restrict__ w,
                                                      const int32_t* __restrict__ long_rows,
                                                      const int32_t* __restrict__ n_long) {
  __shared__ int64_t part[NT / 64];
  const int nl = *n_long;
  for (int i = blockIdx.x; i < nl; i += gridDim.x) {  // block-uniform
    const int32_t x = long_rows[i];
    int64_t sum = 0;
    for (int32_t j = rptr[x] + threadIdx.x; j < rptr[x + 1]; j += NT) sum += len[j];
    sum = wave_sum(sum);
    if (lane_id() == 0) part[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int q = 0; q < NT / 64; ++q) t += part[q];
      w[x - x_lo] = t;
    }
    __syncthreads();
  }
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

// Sorts the rows of [x_lo, x_hi) by their work w into four lists:
//   class 1: w in [1, small_max]           hdr[0], upwards from A
//   class 2: w up to light_max             hdr[1], downwards from A + n
//   class 3: w up to med_max               hdr[2], upwards from B
//   class 4: heavier rows                  hdr[3], downwards from B + n
// small_max <= SMALL_SLOTS / 2, light_max <= LIGHT_MAX and med_max <= MED_MAX
// keep every hash set at most half full (write mode passes the defaults with
// med_max = LIGHT_MAX: no class 3).  A block takes
// CLS_ROWS consecutive rows (CLS_PER per thread), ranks them with one block
// scan and reserves its places with one atomic per class, so few atomics meet
// on the four counters.  In count mode the rows no wave or workgroup hash set
// writes (empty and heavy ones) get count 0 here, before the heavy kernel adds
// to it.
constexpr int CLS_PER = 16;
constexpr int CLS_NT = 1024;  // large blocks: each block reserves list space with one atomic per class
constexpr int CLS_ROWS = CLS_NT * CLS_PER;  // per-class counts of a block fit the 16-bit packed fields

__global__ void __launch_bounds__(CLS_NT) k_classify_rows(int64_t x_lo, int64_t x_hi, const int64_t* __restrict__ w,
                                                      int64_t small_max, int64_t light_max, int64_t med_max,
                                                      int32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ hdr, int32_t* __restrict__ A,
                                                      int32_t* __restrict__ B) {
  __shared__ int64_t wtot[CLS_NT / 64];
  __shared__ int32_t bases[4];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t n = x_hi - x_lo;
  const int64_t r0 = int64_t(blockIdx.x) * CLS_ROWS + int64_t(threadIdx.x) * CLS_PER;
  // classes packed 3 bits per row; per-class counts packed 16 bits each (at most CLS_ROWS)
  uint64_t cls = 0;
  int64_t packed = 0;
#pragma unroll
  for (int k = 0; k < CLS_PER; ++k) {
    const int64_t i = r0 + k;
    int c = 0;
    if (i < n) {
      const int64_t wx = w[i];
      c = wx == 0 ? 0 : wx <= small_max ? 1 : wx <= light_max ? 2 : wx <= med_max ? 3 : 4;
      if (cnt && (c == 0 || c == 4)) cnt[x_lo + i] = 0;
    }
    cls |= uint64_t(c) << (3 * k);
    if (c) packed += int64_t(1) << (16 * (c - 1));
  }
  const int64_t incl = wave_incl_scan(packed);
  if (lane == 63) wtot[wid] = incl;
  __syncthreads();
  int64_t pre = 0, all = 0;
  for (int q = 0; q < CLS_NT / 64; ++q) {
    const int64_t v = wtot[q];
    if (q < wid) pre += v;
    all += v;
  }
  if (threadIdx.x < 4) {
    const int m = int((all >> (16 * threadIdx.x)) & 0xFFFF);
    bases[threadIdx.x] = m ? atomicAdd(&hdr[threadIdx.x], m) : 0;
  }
  __syncthreads();
  const int64_t excl = pre + incl - packed;
  int64_t pos[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) pos[c] = bases[c] + ((excl >> (16 * c)) & 0xFFFF);
#pragma unroll
  for (int k = 0; k < CLS_PER; ++k) {
    const int c = int((cls >> (3 * k)) & 7u);
    const int32_t x = int32_t(x_lo + r0 + k);
    if (c == 1) A[pos[0]++] = x;
    else if (c == 2) A[n - 1 - pos[1]++] = x;
    else if (c == 3) B[pos[2]++] = x;
    else if (c == 4) B[n - 1 - pos[3]++] = x;
  }
}

// The wave's lanes hold up to 64 S segments [s0, s0 + len) (one per join
// key); every z id in them is inserted into the LDS hash set tab of 2^log2t
// slots.  The ids are taken 64 at a time in the order of the segments; lane
// i takes id w0 + i.  Its segment is found without a search: the lanes whose
// (non-empty) segment starts inside the window [w0, w0 + 64) write their lane
// number into the wave's 64-entry LDS array head at that offset, a prefix
// maximum over head carries each owner forward, and a ballot gives the
// segment that covers w0 itself.  head holds -1 on entry and on return.  G
// windows are gathered before inserting.  Returns the number of ids this lane
// inserted first.
template <int G>
__device__ __forceinline__ int hash_insert_segments(int s0, int len, const int32_t* __restrict__ spcol, int32_t* tab,
                                                    int log2t, int32_t* head) {
  const int lane = lane_id();
  const uint32_t tmask = (1u << log2t) - 1u;
  const int incl = wave_scan_add_dpp(len);
  const int excl = incl - len;
  const int total = __builtin_amdgcn_readlane(incl, 63);
  const bool nz = len > 0;
  int fresh = 0;
  for (int t0 = 0; t0 < total; t0 += 64 * G) {
    int32_t zz[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      zz[g] = EMPTY;
      const int w0 = t0 + g * 64;
      if (w0 < total) {
        // w0 < total lies in a non-empty segment starting at or before it
        const uint64_t cov = ballot(nz && excl <= w0);
        const int start = 63 - __builtin_clzll(cov);
        if (nz && excl > w0 && excl < w0 + 64) head[excl - w0] = lane;
        lds_fence();
        int o = head[lane];
        head[lane] = -1;
        o = max(wave_scan_max_dpp(o), start);
        const int os0 = __shfl(s0, o, 64);
        const int oex = __shfl(excl, o, 64);
        const int tt = w0 + lane;
        if (tt < total) zz[g] = spcol[os0 + (tt - oex)];
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int32_t z = zz[g];
      if (z == EMPTY) continue;
      uint32_t h = hash_slot(z, log2t);
      while (true) {
        const int32_t old = atomicCAS(&tab[h], EMPTY, z);
        if (old == EMPTY) {
          ++fresh;
          break;
        }
        if (old == z) break;
        h = (h + 1) & tmask;
      }
    }
  }
  return fresh;
}

// One wavefront per listed row with an LDS hash set of SLOTS slots (at most
// half full: the list holds rows with w <= SLOTS / 2).  A row costs a chain of
// dependent loads (its list entry, row bounds and work, the S segments of its
// join keys, the z ids), so each wave runs a software pipeline over its rows
// r, r + nw, r + 2 nw, ...: while it gathers row r's z ids, the segments of
// row r + nw, the bounds of row r + 2 nw and the list entry of row r + 3 nw are
// in flight.
template <bool WRITE, int SLOTS, int G>
__global__ void __launch_bounds__(NT) k_sparse_light(const int32_t* __restrict__ lst_at, const int32_t* __restrict__ n_ptr,
                                                     int from_end, const int32_t* __restrict__ rptr,
                                                     const int32_t* __restrict__ seg0, const int32_t* __restrict__ seglen,
                                                     const int32_t* __restrict__ spcol, int64_t x_lo,
                                                     const int64_t* __restrict__ w, int32_t* __restrict__ cnt,
                                                     const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ int32_t tab_all[NT / 64][SLOTS];
  __shared__ int32_t head_all[NT / 64][64];
  const int lane = lane_id();
  int32_t* tab = tab_all[threadIdx.x >> 6];
  int32_t* head = head_all[threadIdx.x >> 6];
  head[lane] = -1;
  const int64_t n = *n_ptr;
  const int32_t* lst = from_end ? lst_at - n : lst_at;
  const int64_t nw = (int64_t(gridDim.x) * NT) >> 6;
  int64_t r = (int64_t(blockIdx.x) * NT + threadIdx.x) >> 6;
  const int64_t base_off = WRITE ? off[x_lo] : 0;

  // pipeline registers: c = row r, 1 = row r + nw, 2 = row r + 2 nw
  int xc = r < n ? lst[r] : -1;
  int x1 = r + nw < n ? lst[r + nw] : -1;
  int x2 = r + 2 * nw < n ? lst[r + 2 * nw] : -1;
  int ac = 0, bc = 0, wc = 0;
  if (xc >= 0) {
    ac = rptr[xc];
    bc = rptr[xc + 1];
    wc = int(w[xc - x_lo]);
  }
  int a1 = 0, b1 = 0, w1 = 0;
  if (x1 >= 0) {
    a1 = rptr[x1];
    b1 = rptr[x1 + 1];
    w1 = int(w[x1 - x_lo]);
  }
  int s0c = 0, lc = 0;
  if (ac + lane < bc) {
    s0c = seg0[ac + lane];
    lc = seglen[ac + lane];
  }
  while (xc >= 0) {
    // loads for the rows ahead
    const int x3 = r + 3 * nw < n ? lst[r + 3 * nw] : -1;
    int s01 = 0, l1 = 0;
    if (a1 + lane < b1) {
      s01 = seg0[a1 + lane];
      l1 = seglen[a1 + lane];
    }
    int a2 = 0, b2 = 0, w2 = 0;
    if (x2 >= 0) {
      a2 = rptr[x2];
      b2 = rptr[x2 + 1];
      w2 = int(w[x2 - x_lo]);
    }

    // row r
    int log2t = 6;
    while ((1 << log2t) < 2 * wc) ++log2t;
    const int t = 1 << log2t;
    for (int i = lane; i < t; i += 64) tab[i] = EMPTY;
    lds_fence();
    int fresh = hash_insert_segments<G>(s0c, lc, spcol, tab, log2t, head);
    for (int c0 = ac + 64; c0 < bc; c0 += 64) {
      const int j = c0 + lane;
      int s0 = 0, len = 0;
      if (j < bc) {
        s0 = seg0[j];
        len = seglen[j];
      }
      fresh += hash_insert_segments<G>(s0, len, spcol, tab, log2t, head);
    }
    const int count = wave_sum(fresh);
    if (!WRITE) {
      if (lane == 0) cnt[xc] = count;
    } else {
      lds_fence();
      wave_bitonic(tab, t);
      int32_t* dst = out + (off[xc] - base_off);
      for (int i = lane; i < count; i += 64) dst[i] = tab[i];
    }
    lds_fence();

    r += nw;
    xc = x1;
    ac = a1;
    bc = b1;
    wc = w1;
    s0c = s01;
    lc = l1;
    x1 = x2;
    a1 = a2;
    b1 = b2;
    w1 = w2;
    x2 = x3;
  }
}

// count mode, rows with LIGHT_MAX < w <= MED_MAX: one workgroup per row and
// one LDS hash set of the row's z ids (at most half full) shared by its waves;
// each wave takes 64 join keys of the row at a time
__global__ void __launch_bounds__(NT) k_sparse_medium_count(const int32_t* __restrict__ lst, const int32_t* __restrict__ n_ptr,
                                                            const int32_t* __restrict__ rptr,
                                                            const int32_t* __restrict__ seg0,
                                                            const int32_t* __restrict__ seglen,
                                                            const int32_t* __restrict__ spcol, int64_t x_lo,
                                                            const int64_t* __restrict__ w, int32_t* __restrict__ cnt) {
  __shared__ int32_t tab[2 * MED_MAX];
  __shared__ int32_t head_all[NT / 64][64];
  __shared__ int red[NT / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  int32_t* head = head_all[wid];
  head[lane] = -1;
  const int n = *n_ptr;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int x = lst[i];
    const int wx = int(w[x - x_lo]);
    const int a = rptr[x], b = rptr[x + 1];
    int log2t = 6;
    while ((1 << log2t) < 2 * wx) ++log2t;
    const int t = 1 << log2t;
    for (int k = threadIdx.x; k < t; k += NT) tab[k] = EMPTY;
    __syncthreads();
    int fresh = 0;
    for (int c0 = a + wid * 64; c0 < b; c0 += NT) {
      const int j = c0 + lane;
      int s0 = 0, len = 0;
      if (j < b) {
        s0 = seg0[j];
        len = seglen[j];
      }
      fresh += hash_insert_segments<4>(s0, len, spcol, tab, log2t, head);
    }
    const int c = wave_sum(fresh);
    if (lane == 0) red[wid] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int q = 0; q < NT / 64; ++q) tot += red[q];
      cnt[x] = tot;
    }
    __syncthreads();
  }
}

// count mode: one workgroup per (heavy row, window blockIdx.y)
__global__ void __launch_bounds__(NT) k_sparse_heavy_count(const int32_t* __restrict__ rptr,
                                                           const int32_t* __restrict__ seg0,
                                                           const int32_t* __restrict__ seglen,
                                                           const int32_t* __restrict__ spcol, int n_inst,
                                                           const int32_t* __restrict__ x_base,
                                                           const int32_t* __restrict__ z_base,
                                                           const int32_t* __restrict__ lst_end,
                                                           const int32_t* __restrict__ n_list,
                                                           int32_t* __restrict__ cnt) {
  __shared__ uint32_t bm[HB_WORDS];
  __shared__ int red[NT / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int nh = *n_list;
  const int32_t* list = lst_end - nh;
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
                                                           const int32_t* __restrict__ lst_end,
                                                           const int32_t* __restrict__ n_list,
                                                           const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ uint32_t bm[HB_WORDS];
  __shared__ int red[NT / 64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int64_t base_off = off[x_lo];
  const int nh = *n_list;
  const int32_t* list = lst_end - nh;

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
  const int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  const int64_t ne = j_hi - j_lo;
  if (ne > 0) {
    hipLaunchKernelGGL(k_entry_seg, dim3(chunk_grid(ne)), dim3(NT), 0, s, c.rcol, c.spptr, j_lo, j_hi, seg0, seglen);
    JP_LAUNCH_CHECK();
  }
  int32_t* n_long = a.alloc<int32_t>(1, s);
  int32_t* long_rows = a.alloc<int32_t>(std::max<int64_t>(std::min<int64_t>(n, ne / ROW_LONG + 1), 1), s);
  fill_i32(n_long, 1, 0, s);
  const int g = int(std::min<int64_t>((n + NT - 1) / NT, 1 << 16));
  hipLaunchKernelGGL(k_row_work, dim3(g), dim3(NT), 0, s, c.rptr, seglen, x_lo, x_hi, w, long_rows, n_long);
  hipLaunchKernelGGL(k_row_work_long, dim3(int(std::min<int64_t>(n, 1024))), dim3(NT), 0, s, c.rptr, seglen, x_lo, w,
                     (const int32_t*)long_rows, (const int32_t*)n_long);
  JP_LAUNCH_CHECK();
  a.give_back(long_rows, s);
  a.give_back(n_long, s);
}

int64_t sparse_list_ints(int64_t n_rows) { return 2 * n_rows + 4; }

void sparse_bmm(const RowCtx& c, int64_t x_lo, int64_t x_hi, const int64_t* w, int32_t* cnt, const int64_t* off,
                int32_t* out, int32_t* lists, hipStream_t s) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  // lists: 4 header ints (the list lengths), then regions A (light rows) and
  // B (medium and heavy rows) of n ints, each holding two lists from both ends
  int32_t* hdr = lists;
  int32_t* A = lists + 4;
  int32_t* B = A + n;
  fill_i32(hdr, 4, 0, s);
  // count mode takes the plan's class bounds (tuned or pinned), write mode the defaults
  const int64_t light_max = out ? LIGHT_MAX : std::min<int64_t>(LIGHT_MAX, c.light_max > 0 ? c.light_max : LIGHT_MAX);
  const int64_t small_max = std::min<int64_t>(SMALL_SLOTS / 2, light_max);
  const int64_t med_max =
      out ? LIGHT_MAX : std::max<int64_t>(light_max, std::min<int64_t>(MED_MAX, c.med_max > 0 ? c.med_max : MED_MAX));
  hipLaunchKernelGGL(k_classify_rows, dim3(int((n + CLS_ROWS - 1) / CLS_ROWS)), dim3(CLS_NT), 0, s, x_lo, x_hi, w,
                     small_max, light_max, med_max, cnt, hdr, A, B);
  JP_LAUNCH_CHECK();
  // light rows: four times as many waves as stay resident (8 blocks of 4 waves
  // per CU with 512-slot tables, 5 with 2048), each pipelining over its rows
  const int gs = int(std::min<int64_t>((n + 3) / 4, 8192));
  const int gb = int(std::min<int64_t>((n + 3) / 4, 5120));
  const int gh = int(std::min<int64_t>(n, 1024));
  if (out) {
    hipLaunchKernelGGL((k_sparse_light<true, SMALL_SLOTS, 4>), dim3(gs), dim3(NT), 0, s, A, hdr + 0, 0, c.rptr, c.seg0,
                       c.seglen, c.spcol, x_lo, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sparse_light<true, HT_SLOTS, 4>), dim3(gb), dim3(NT), 0, s, A + n, hdr + 1, 1, c.rptr, c.seg0,
                       c.seglen, c.spcol, x_lo, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sparse_heavy_write, dim3(gh), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen, c.spcol, c.n_inst,
                       c.x_base, c.z_base, x_lo, B + n, hdr + 3, off, out);
    JP_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL((k_sparse_light<false, SMALL_SLOTS, 4>), dim3(gs), dim3(NT), 0, s, A, hdr + 0, 0, c.rptr, c.seg0,
                       c.seglen, c.spcol, x_lo, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_sparse_light<false, HT_SLOTS, 4>), dim3(gb), dim3(NT), 0, s, A + n, hdr + 1, 1, c.rptr,
                       c.seg0, c.seglen, c.spcol, x_lo, w, cnt, off, out);
    JP_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sparse_medium_count, dim3(gh), dim3(NT), 0, s, B, hdr + 2, c.rptr, c.seg0, c.seglen, c.spcol,
                       x_lo, w, cnt);
    JP_LAUNCH_CHECK();
    const int wins = int(std::max<int64_t>(1, (c.max_z_range + HB_BITS - 1) / HB_BITS));
    hipLaunchKernelGGL(k_sparse_heavy_count, dim3(gh, wins), dim3(NT), 0, s, c.rptr, c.seg0, c.seglen, c.spcol,
                       c.n_inst, c.x_base, c.z_base, B + n, hdr + 3, cnt);
    JP_LAUNCH_CHECK();
  }
}

}  // namespace jp
