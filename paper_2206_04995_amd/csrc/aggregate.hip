// Join-Aggregate (paper Sec. 4.1, group-by attributes from both tables):
//   G_{x,z} COUNT(*), SUM(R.v * S.u)  over  R(x, y, v) JOIN_y S(z, y, u).
// The groups are the Join-Project result; each carries the number of its join
// rows and the sum of v * u over them (int64, wrapping).
//
// As the paper adapts DIM^3, the deduplicating accumulator of each x row (the
// SPA of SparseBMM) becomes an aggregate accumulator, and the dense part
// becomes a plain dense accumulation:
// * rows with little work (w = join rows of the row <= LIGHT_W) run one per
//   wavefront with an LDS hash map z -> (count, sum); the write pass sorts the
//   row's groups by z with a bitonic sort in LDS;
// * heavier rows run per window of WZ z ids with dense LDS arrays count[WZ]
//   and sum[WZ] indexed by z (a presence bitmap in the count pass), and emit
//   each window in z order.
// The mapping is this path's own: S sorted by (y, z) and R by x (radix sorts
// of the tuple indices), order-preserving z ids, join keys of R found in S's
// distinct y by binary search.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/jp.h"
#include "common.h"
#include "plan_impl.h"
#include "pool.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

constexpr int NT = 256;
constexpr int LIGHT_W = 512;      // rows with at most this many join rows use a wave hash map
constexpr int LSLOTS = 1024;      // its slots (load <= 1/2)
constexpr int LWAVES = 2;         // waves per workgroup of the light kernel
constexpr int WZ = 8192;          // z ids per window of the heavy kernels
constexpr int32_t EMPTY = 0x7FFFFFFF;

inline int grid(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 1 << 20))); }

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t hslot(int32_t z) { return (uint32_t(z) * 0x9E3779B1u) >> (32 - 10); }

// block-wide exclusive scan of one int per thread (NT threads); *total = the sum
__device__ int block_excl_scan_i32(int v, int* lds, int& total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int incl = wave_incl_scan(v);
  if (lane == 63) lds[wid] = incl;
  __syncthreads();
  int pre = 0;
  total = 0;
  for (int q = 0; q < NT / 64; ++q) {
    const int t = lds[q];
    if (q < wid) pre += t;
    total += t;
  }
  __syncthreads();
  return pre + incl - v;
}

// ------------------------------------------------------------ mapping helpers

__global__ void k_iota(uint32_t* __restrict__ p, int64_t n) {
  GRID_STRIDE(i, n) { p[i] = uint32_t(i); }
}

// keys[i] = v[perm[i]] - mn (perm null: identity)
__global__ void k_keys(const int32_t* __restrict__ v, const uint32_t* __restrict__ perm, int64_t n, int32_t mn,
                       uint32_t* __restrict__ keys) {
  GRID_STRIDE(i, n) { keys[i] = uint32_t(int64_t(v[perm ? perm[i] : i]) - int64_t(mn)); }
}

// zid[perm[p]] = id of sorted position p (E from run ids)
__global__ void k_scatter_ids(const uint32_t* __restrict__ perm, const int32_t* __restrict__ E, int64_t n,
                              int32_t* __restrict__ zid) {
  GRID_STRIDE(p, n) { zid[perm[p]] = E[p + 1] - 1; }
}

// S in (y, z) order: z id and u of each position
__global__ void k_gather_s(const uint32_t* __restrict__ perm, int64_t n, const int32_t* __restrict__ zid,
                           const int32_t* __restrict__ su, int32_t* __restrict__ s_z, int32_t* __restrict__ s_u) {
  GRID_STRIDE(p, n) {
    const uint32_t i = perm[p];
    s_z[p] = zid[i];
    s_u[p] = su[i];
  }
}

// R in x order: y id (-1: no partner) and v of each position, and its number of join rows
__global__ void k_gather_r(const uint32_t* __restrict__ perm, int64_t n, const int32_t* __restrict__ yid,
                           const int32_t* __restrict__ rv, const int32_t* __restrict__ sptr, int32_t* __restrict__ r_y,
                           int32_t* __restrict__ r_v, int32_t* __restrict__ deg) {
  GRID_STRIDE(p, n) {
    const uint32_t i = perm[p];
    const int32_t y = yid[i];
    r_y[p] = y;
    r_v[p] = rv[i];
    deg[p] = y >= 0 ? sptr[y + 1] - sptr[y] : 0;
  }
}

// the rows with more than LIGHT_W join rows (the heavy list, any order);
// every count starts at 0
__global__ void k_agg_classify(const int32_t* __restrict__ rptr, const int64_t* __restrict__ wpre, int64_t nx,
                               int32_t* __restrict__ cnt, int32_t* __restrict__ n_heavy, int32_t* __restrict__ heavy) {
  GRID_STRIDE(x, nx) {
    cnt[x] = 0;
    if (wpre[rptr[x + 1]] - wpre[rptr[x]] > LIGHT_W) heavy[atomicAdd(n_heavy, 1)] = int32_t(x);
  }
}

// ------------------------------------------------------------ light rows

struct AggCtx {
  const int32_t *rptr, *r_y, *r_v, *sptr, *s_z, *s_u, *vals_x, *vals_z;
  const int64_t* wpre;
  int64_t nz;
};

// the join row t of row entries [a, b): the entry p and the S position
__device__ __forceinline__ void join_row(const AggCtx& c, int a, int b, int64_t w0, int64_t t, int& p, int& sp) {
  int lo = a, hi = b - 1;  // last p with wpre[p] - w0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (c.wpre[mid] - w0 <= t) lo = mid;
    else hi = mid - 1;
  }
  p = lo;
  sp = c.sptr[c.r_y[p]] + int(t - (c.wpre[p] - w0));
}

// one wave per row of [x_lo, x_hi) with 1 <= w <= LIGHT_W (other rows are skipped)
template <bool WRITE>
__global__ void __launch_bounds__(64 * LWAVES) k_agg_light(AggCtx c, int64_t x_lo, int64_t x_hi,
                                                           int32_t* __restrict__ cnt, const int64_t* __restrict__ goff,
                                                           int64_t g_lo, int64_t g_hi, int32_t* __restrict__ ox,
                                                           int32_t* __restrict__ oz, int64_t* __restrict__ ocnt,
                                                           int64_t* __restrict__ osum) {
  __shared__ int32_t tkey_all[LWAVES][LSLOTS];
  __shared__ int32_t tcnt_all[LWAVES][LSLOTS];
  __shared__ unsigned long long tsum_all[LWAVES][LSLOTS];
  __shared__ int32_t skey_all[WRITE ? LWAVES : 1][WRITE ? LIGHT_W : 1];
  __shared__ int32_t sidx_all[WRITE ? LWAVES : 1][WRITE ? LIGHT_W : 1];
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  int32_t* tkey = tkey_all[wid];
  int32_t* tcnt = tcnt_all[wid];
  unsigned long long* tsum = tsum_all[wid];
  for (int64_t x = x_lo + int64_t(blockIdx.x) * LWAVES + wid; x < x_hi; x += int64_t(gridDim.x) * LWAVES) {
    const int a = c.rptr[x], b = c.rptr[x + 1];
    const int64_t w0 = c.wpre[a];
    const int64_t wl = c.wpre[b] - w0;
    if (wl == 0 || wl > LIGHT_W) continue;
    const int w = int(wl);
    for (int i = lane; i < LSLOTS; i += 64) {
      tkey[i] = EMPTY;
      tcnt[i] = 0;
      tsum[i] = 0ull;
    }
    wave_sync();
    int fresh = 0;
    for (int t = lane; t < w; t += 64) {
      int p, sp;
      join_row(c, a, b, w0, t, p, sp);
      const int32_t z = c.s_z[sp];
      const int64_t vu = int64_t(c.r_v[p]) * int64_t(c.s_u[sp]);
      uint32_t h = hslot(z);
      while (true) {
        const int32_t old = atomicCAS(&tkey[h], EMPTY, z);
        if (old == EMPTY) ++fresh;
        if (old == EMPTY || old == z) break;
        h = (h + 1) & (LSLOTS - 1);
      }
      atomicAdd(&tcnt[h], 1);
      atomicAdd(&tsum[h], (unsigned long long)vu);
    }
    wave_sync();
    if (!WRITE) {
      const int tot = wave_sum(fresh);
      if (lane == 0) cnt[x] = tot;
      continue;
    }
    // write: the row's groups in z order
    int32_t* skey = skey_all[wid];
    int32_t* sidx = sidx_all[wid];
    int k = 0;
    for (int s0 = 0; s0 < LSLOTS; s0 += 64) {
      const bool occ = tkey[s0 + lane] != EMPTY;
      const uint64_t m = ballot(occ);
      if (occ) {
        const int pos = k + __popcll(m & lanemask_lt());
        skey[pos] = tkey[s0 + lane];
        sidx[pos] = s0 + lane;
      }
      k += __popcll(m);
    }
    int P = 1;
    while (P < k) P <<= 1;
    for (int i = k + lane; i < P; i += 64) {
      skey[i] = EMPTY;
      sidx[i] = 0;
    }
    wave_sync();
    for (int kk = 2; kk <= P; kk <<= 1) {
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int i = lane; i < P; i += 64) {
          const int l = i ^ j;
          if (l > i) {
            const bool up = (i & kk) == 0;
            const int32_t u = skey[i], v = skey[l];
            if ((u > v) == up) {
              skey[i] = v;
              skey[l] = u;
              const int32_t t2 = sidx[i];
              sidx[i] = sidx[l];
              sidx[l] = t2;
            }
          }
        }
        wave_sync();
      }
    }
    const int64_t g0 = goff[x];
    const int32_t xv = c.vals_x[x];
    for (int i = lane; i < k; i += 64) {
      const int64_t g = g0 + i;
      if (g < g_lo || g >= g_hi) continue;
      const int slot = sidx[i];
      ox[g - g_lo] = xv;
      oz[g - g_lo] = c.vals_z[skey[i]];
      ocnt[g - g_lo] = tcnt[slot];
      osum[g - g_lo] = int64_t(tsum[slot]);
    }
    wave_sync();
  }
}

// ------------------------------------------------------------ heavy rows

// the part [lo, hi) of S row y whose z ids lie in [zlo, zhi)
__device__ __forceinline__ void window_part(const AggCtx& c, int32_t y, int32_t zlo, int32_t zhi, int& lo, int& hi) {
  const int s0 = c.sptr[y], s1 = c.sptr[y + 1];
  lo = int(lower_bound_dev<int32_t>(c.s_z, s0, s1, zlo));
  hi = int(lower_bound_dev<int32_t>(c.s_z, lo, s1, zhi));
}

// count pass: one workgroup per (heavy row, window): distinct z of the window
__global__ void __launch_bounds__(NT) k_agg_heavy_count(AggCtx c, const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ n_list, int32_t* __restrict__ cnt) {
  __shared__ uint32_t bm[WZ / 32];
  __shared__ int part[NT / 64];
  const int nl = *n_list;
  const int nwin = int((c.nz + WZ - 1) / WZ);
  for (int64_t item = blockIdx.x; item < int64_t(nl) * nwin; item += gridDim.x) {
    const int x = list[item / nwin];
    const int32_t zlo = int32_t((item % nwin) * WZ), zhi = zlo + WZ;
    for (int i = threadIdx.x; i < WZ / 32; i += NT) bm[i] = 0u;
    __syncthreads();
    const int a = c.rptr[x], b = c.rptr[x + 1];
    for (int p = a + threadIdx.x; p < b; p += NT) {
      const int32_t y = c.r_y[p];
      if (y < 0) continue;
      int lo, hi;
      window_part(c, y, zlo, zhi, lo, hi);
      for (int q = lo; q < hi; ++q) {
        const int d = c.s_z[q] - zlo;
        atomicOr(&bm[d >> 5], 1u << (d & 31));
      }
    }
    __syncthreads();
    int pc = 0;
    for (int i = threadIdx.x; i < WZ / 32; i += NT) pc += __popc(bm[i]);
    pc = wave_sum(pc);
    if (lane_id() == 0) part[threadIdx.x >> 6] = pc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int q = 0; q < NT / 64; ++q) t += part[q];
      if (t) atomicAdd(&cnt[x], t);
    }
    __syncthreads();
  }
}

// write pass: one workgroup per heavy row, its windows in order with dense
// LDS accumulators; groups outside [g_lo, g_hi) are skipped
__global__ void __launch_bounds__(NT) k_agg_heavy_write(AggCtx c, const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ n_list, int64_t x_lo, int64_t x_hi,
                                                        const int64_t* __restrict__ goff, int64_t g_lo, int64_t g_hi,
                                                        int32_t* __restrict__ ox, int32_t* __restrict__ oz,
                                                        int64_t* __restrict__ ocnt, int64_t* __restrict__ osum) {
  __shared__ int32_t acnt[WZ];
  __shared__ unsigned long long asum[WZ];
  __shared__ int32_t scan_lds[NT / 64];
  constexpr int PER = WZ / NT;  // z ids per thread in the emit step
  const int nl = *n_list;
  const int nwin = int((c.nz + WZ - 1) / WZ);
  for (int r = blockIdx.x; r < nl; r += gridDim.x) {
    const int x = list[r];
    if (x < x_lo || x >= x_hi) continue;
    const int a = c.rptr[x], b = c.rptr[x + 1];
    const int32_t xv = c.vals_x[x];
    int64_t g = goff[x];
    if (goff[x + 1] <= g_lo || g >= g_hi) continue;  // no group of this row is asked for
    for (int win = 0; win < nwin; ++win) {
      const int32_t zlo = win * WZ, zhi = zlo + WZ;
      for (int i = threadIdx.x; i < WZ; i += NT) {
        acnt[i] = 0;
        asum[i] = 0ull;
      }
      __syncthreads();
      for (int p = a + threadIdx.x; p < b; p += NT) {
        const int32_t y = c.r_y[p];
        if (y < 0) continue;
        const int64_t v = c.r_v[p];
        int lo, hi;
        window_part(c, y, zlo, zhi, lo, hi);
        for (int q = lo; q < hi; ++q) {
          const int d = c.s_z[q] - zlo;
          atomicAdd(&acnt[d], 1);
          atomicAdd(&asum[d], (unsigned long long)(v * int64_t(c.s_u[q])));
        }
      }
      __syncthreads();
      int mine = 0;
      for (int k = 0; k < PER; ++k) mine += acnt[threadIdx.x * PER + k] ? 1 : 0;
      int total;
      int pos = block_excl_scan_i32(mine, scan_lds, total);
      for (int k = 0; k < PER; ++k) {
        const int d = threadIdx.x * PER + k;
        if (acnt[d]) {
          const int64_t gg = g + pos;
          if (gg >= g_lo && gg < g_hi) {
            ox[gg - g_lo] = xv;
            oz[gg - g_lo] = c.vals_z[zlo + d];
            ocnt[gg - g_lo] = acnt[d];
            osum[gg - g_lo] = int64_t(asum[d]);
          }
          ++pos;
        }
      }
      g += total;
      __syncthreads();
    }
  }
}

// rows[0] = first row with goff[row + 1] > g0, rows[1] = first row with goff[row] >= g1
__global__ void k_agg_rows(const int64_t* __restrict__ goff, int64_t nx, int64_t g0, int64_t g1,
                           int64_t* __restrict__ rows) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t lo = 0, hi = nx;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (goff[m + 1] <= g0) lo = m + 1;
    else hi = m;
  }
  rows[0] = lo;
  lo = 0;
  hi = nx;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (goff[m] < g1) lo = m + 1;
    else hi = m;
  }
  rows[1] = lo;
}

void lc() { JP_LAUNCH_CHECK(); }



struct AggPlan {
  Budget B;
  Arena A{&B};
  hipStream_t stream = nullptr;
  int64_t nr = 0, ns = 0, NX = 0, NY = 0, NZ = 0, out_j = 0, groups = 0;
  int32_t *rptr = nullptr, *r_y = nullptr, *r_v = nullptr, *sptr = nullptr, *s_z = nullptr, *s_u = nullptr;
  int32_t *vals_x = nullptr, *vals_z = nullptr, *cnt = nullptr, *heavy = nullptr, *n_heavy = nullptr;
  int64_t *wpre = nullptr, *goff = nullptr;
  bool executed = false, have_groups = false;

  AggCtx ctx() const { return AggCtx{rptr, r_y, r_v, sptr, s_z, s_u, vals_x, vals_z, wpre, NZ}; }

  // sort of the values v[perm[i]] - mn by LSD radix, carrying perm; returns the sorted (keys, perm)
  void sort_by(const int32_t* v, int64_t n, int32_t mn, int32_t mx, uint32_t*& keys, uint32_t*& perm,
               uint32_t*& keys2, uint32_t*& perm2, Arena& T, hipStream_t s) {
    hipLaunchKernelGGL(k_keys, dim3(grid(n)), dim3(NT), 0, s, v, perm, n, mn, keys);
    lc();
    const int bits = mn < mx ? bits_for(uint64_t(int64_t(mx) - int64_t(mn) + 1)) : 0;
    if (bits > 0 && radix_sort_pairs(keys, perm, keys2, perm2, n, bits, s, T)) {
      std::swap(keys, keys2);
      std::swap(perm, perm2);
    }
  }

  void build(const int32_t* rx, const int32_t* ry, const int32_t* rv, int64_t nr_, const int32_t* sz,
             const int32_t* sy, const int32_t* su, int64_t ns_, hipStream_t s) {
    stream = s;
    nr = nr_;
    ns = ns_;
    Arena T(&B);
    const int64_t NRa = std::max<int64_t>(nr, 1), NSa = std::max<int64_t>(ns, 1);
    int32_t* bases = T.alloc<int32_t>(4, s);
    const int32_t hb[4] = {0, int32_t(nr), 0, int32_t(ns)};
    JP_HIP(hipMemcpyAsync(bases, hb, sizeof(hb), hipMemcpyHostToDevice, s));
    int32_t* mm = T.alloc<int32_t>(6, s);
    seg_minmax(sz, ns, bases + 2, 1, mm + 0, mm + 1, s);
    seg_minmax(sy, ns, bases + 2, 1, mm + 2, mm + 3, s);
    seg_minmax(rx, nr, bases, 1, mm + 4, mm + 5, s);
    int32_t h[6];
    JP_HIP(hipMemcpyAsync(h, mm, sizeof(h), hipMemcpyDeviceToHost, s));
    JP_HIP(hipStreamSynchronize(s));
    // single-instance key layouts for run_ids: koff = {0, range}, mn
    int64_t* koff = T.alloc<int64_t>(6, s);
    const int64_t hk[6] = {0, ns ? int64_t(h[1]) - h[0] + 1 : 0, 0, ns ? int64_t(h[3]) - h[2] + 1 : 0,
                           0, nr ? int64_t(h[5]) - h[4] + 1 : 0};
    JP_HIP(hipMemcpyAsync(koff, hk, sizeof(hk), hipMemcpyHostToDevice, s));
    int32_t* mns = T.alloc<int32_t>(3, s);
    const int32_t hm[3] = {h[0], h[2], h[4]};
    JP_HIP(hipMemcpyAsync(mns, hm, sizeof(hm), hipMemcpyHostToDevice, s));

    // S by z: z ids (order preserving) and their values
    uint32_t* k1 = T.alloc<uint32_t>(NSa, s);
    uint32_t* p1 = T.alloc<uint32_t>(NSa, s);
    uint32_t* k2 = T.alloc<uint32_t>(NSa, s);
    uint32_t* p2 = T.alloc<uint32_t>(NSa, s);
    hipLaunchKernelGGL(k_iota, dim3(grid(ns)), dim3(NT), 0, s, p1, ns);
    lc();
    int32_t* E = T.alloc<int32_t>(ns + 1, s);
    int32_t* first = T.alloc<int32_t>(ns + 1, s);
    vals_z = A.alloc<int32_t>(NSa, s);
    int32_t* zid = T.alloc<int32_t>(NSa, s);
    if (ns) {
      sort_by(sz, ns, h[0], h[1], k1, p1, k2, p2, T, s);
      run_ids(k1, ns, koff, mns, 1, E, first, vals_z, s, T);
      hipLaunchKernelGGL(k_scatter_ids, dim3(grid(ns)), dim3(NT), 0, s, p1, E, ns, zid);
      lc();
    } else {
      fill_i32(E, 1, 0, s);
    }
    int32_t nz = 0;
    JP_HIP(hipMemcpyAsync(&nz, E + ns, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    // S by (y, z): a stable sort by y of the z order; CSR by y
    int32_t* Ey = T.alloc<int32_t>(ns + 1, s);
    sptr = A.alloc<int32_t>(ns + 1, s);
    int32_t* vals_y = T.alloc<int32_t>(NSa, s);
    s_z = A.alloc<int32_t>(NSa, s);
    s_u = A.alloc<int32_t>(NSa, s);
    if (ns) {
      sort_by(sy, ns, h[2], h[3], k1, p1, k2, p2, T, s);
      run_ids(k1, ns, koff + 2, mns + 1, 1, Ey, sptr, vals_y, s, T);
      hipLaunchKernelGGL(k_gather_s, dim3(grid(ns)), dim3(NT), 0, s, p1, ns, zid, su, s_z, s_u);
      lc();
    } else {
      fill_i32(Ey, 1, 0, s);
      fill_i32(sptr, 1, 0, s);
    }
    int32_t* y_base = T.alloc<int32_t>(2, s);
    gather_bases(Ey, bases + 2, 1, y_base, s);
    // R: join key ids by binary search in S's distinct y; R by x
    int32_t* keep = T.alloc<int32_t>(NRa, s);
    int32_t* yid = T.alloc<int32_t>(NRa, s);
    semijoin(ry, nr, bases, 1, vals_y, y_base, keep, yid, s);
    uint32_t* q1 = T.alloc<uint32_t>(NRa, s);
    uint32_t* r1 = T.alloc<uint32_t>(NRa, s);
    uint32_t* q2 = T.alloc<uint32_t>(NRa, s);
    uint32_t* r2 = T.alloc<uint32_t>(NRa, s);
    hipLaunchKernelGGL(k_iota, dim3(grid(nr)), dim3(NT), 0, s, r1, nr);
    lc();
    int32_t* Ex = T.alloc<int32_t>(nr + 1, s);
    rptr = A.alloc<int32_t>(nr + 1, s);
    vals_x = A.alloc<int32_t>(NRa, s);
    r_y = A.alloc<int32_t>(NRa, s);
    r_v = A.alloc<int32_t>(NRa, s);
    int32_t* deg = T.alloc<int32_t>(NRa, s);
    if (nr) {
      sort_by(rx, nr, h[4], h[5], q1, r1, q2, r2, T, s);
      run_ids(q1, nr, koff + 4, mns + 2, 1, Ex, rptr, vals_x, s, T);
      hipLaunchKernelGGL(k_gather_r, dim3(grid(nr)), dim3(NT), 0, s, r1, nr, yid, rv, sptr, r_y, r_v, deg);
      lc();
    } else {
      fill_i32(Ex, 1, 0, s);
      fill_i32(rptr, 1, 0, s);
    }
    wpre = A.alloc<int64_t>(nr + 1, s);
    scan_excl_i32_to_i64(deg, wpre, nr, s, T);
    int32_t nx = 0;
    JP_HIP(hipMemcpyAsync(&nx, Ex + nr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    int32_t ny = 0;
    JP_HIP(hipMemcpyAsync(&ny, Ey + ns, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JP_HIP(hipMemcpyAsync(&out_j, wpre + nr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JP_HIP(hipStreamSynchronize(s));
    NX = nx;
    NY = ny;
    NZ = nz;
    T.release(s);
  }

  void execute(hipStream_t s) {
    if (!cnt) {
      cnt = A.alloc<int32_t>(std::max<int64_t>(NX, 1), s);
      heavy = A.alloc<int32_t>(std::max<int64_t>(NX, 1), s);
      n_heavy = A.alloc<int32_t>(1, s);
      goff = A.alloc<int64_t>(NX + 1, s);
    }
    fill_i32(n_heavy, 1, 0, s);
    Arena T(&B);
    if (NX) {
      hipLaunchKernelGGL(k_agg_classify, dim3(grid(NX)), dim3(NT), 0, s, rptr, wpre, NX, cnt, n_heavy, heavy);
      lc();
      const AggCtx c = ctx();
      const int lg = int(std::min<int64_t>((NX + LWAVES - 1) / LWAVES, 1 << 16));
      hipLaunchKernelGGL(k_agg_light<false>, dim3(lg), dim3(64 * LWAVES), 0, s, c, int64_t(0), NX, cnt,
                         (const int64_t*)nullptr, int64_t(0), int64_t(0), (int32_t*)nullptr, (int32_t*)nullptr,
                         (int64_t*)nullptr, (int64_t*)nullptr);
      lc();
      hipLaunchKernelGGL(k_agg_heavy_count, dim3(4096), dim3(NT), 0, s, c, heavy, n_heavy, cnt);
      lc();
    }
    scan_excl_i32_to_i64(cnt, goff, NX, s, T);
    T.release(s);
    executed = true;
    have_groups = false;
  }

  void fetch_groups(hipStream_t s) {
    if (!executed) throw Error(JP_ESTATE, "group count before execute");
    if (have_groups) return;
    JP_HIP(hipMemcpyAsync(&groups, goff + NX, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    JP_HIP(hipStreamSynchronize(s));
    have_groups = true;
  }

  int64_t materialize(int64_t first, int64_t maxg, int32_t* ox, int32_t* oz, int64_t* ocnt, int64_t* osum,
                      hipStream_t s) {
    fetch_groups(s);
    if (first > groups) throw Error(JP_ERANGE, "first beyond the number of groups");
    const int64_t nw = std::min(maxg, groups - first);
    if (nw <= 0) return 0;
    const int64_t g0 = first, g1 = first + nw;
    Arena T(&B);
    int64_t* rows = T.alloc<int64_t>(2, s);
    hipLaunchKernelGGL(k_agg_rows, dim3(1), dim3(64), 0, s, goff, NX, g0, g1, rows);
    lc();
    int64_t hr[2];
    JP_HIP(hipMemcpyAsync(hr, rows, sizeof(hr), hipMemcpyDeviceToHost, s));
    JP_HIP(hipStreamSynchronize(s));
    const int64_t xl = hr[0], xh = hr[1];
    const AggCtx c = ctx();
    const int lg = int(std::max<int64_t>(1, std::min<int64_t>((xh - xl + LWAVES - 1) / LWAVES, 1 << 16)));
    hipLaunchKernelGGL(k_agg_light<true>, dim3(lg), dim3(64 * LWAVES), 0, s, c, xl, xh, cnt, (const int64_t*)goff, g0,
                       g1, ox, oz, ocnt, osum);
    lc();
    hipLaunchKernelGGL(k_agg_heavy_write, dim3(1024), dim3(NT), 0, s, c, heavy, n_heavy, xl, xh, (const int64_t*)goff,
                       g0, g1, ox, oz, ocnt, osum);
    lc();
    JP_HIP(hipStreamSynchronize(s));
    T.release(s);
    return nw;
  }

  ~AggPlan() { A.release(stream); }
};

jp_status afail(int st, const std::string& m) {
  set_last_error(m);
  return jp_status(st);
}

template <class F>
jp_status aguard(F&& f) {
  try {
    f();
    return JP_OK;
  } catch (const Error& e) {
    return afail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return afail(JP_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return afail(JP_EHIP, e.what());
  }
}

}  // namespace
}  // namespace jp

struct jp_agg {
  jp::AggPlan p;
};

extern "C" {

jp_status jp_agg_create(const int32_t* r_x, const int32_t* r_y, const int32_t* r_v, int64_t n_r, const int32_t* s_z,
                        const int32_t* s_y, const int32_t* s_u, int64_t n_s, hipStream_t stream, jp_agg** out) {
  using jp::afail;
  if (!out) return afail(JP_EINVAL, "out is null");
  *out = nullptr;
  if (n_r < 0 || n_s < 0) return afail(JP_EINVAL, "negative tuple count");
  if (n_r > INT32_MAX || n_s > INT32_MAX) return afail(JP_EINVAL, "more than 2^31-1 tuples");
  if ((n_r > 0 && (!r_x || !r_y || !r_v)) || (n_s > 0 && (!s_z || !s_y || !s_u)))
    return afail(JP_EINVAL, "null column with n > 0");
  jp_agg* a = new (std::nothrow) jp_agg();
  if (!a) return afail(JP_ENOMEM, "host allocation failed");
  jp_status st = jp::aguard([&] { a->p.build(r_x, r_y, r_v, n_r, s_z, s_y, s_u, n_s, stream); });
  if (st != JP_OK) {
    (void)hipStreamSynchronize(stream);
    delete a;
    return st;
  }
  *out = a;
  return JP_OK;
}

jp_status jp_agg_execute(jp_agg* a, hipStream_t stream) {
  if (!a) return jp::afail(JP_EINVAL, "null aggregate");
  return jp::aguard([&] { a->p.execute(stream); });
}

jp_status jp_agg_count(jp_agg* a, int64_t* groups, int64_t* out_j, hipStream_t stream) {
  if (!a) return jp::afail(JP_EINVAL, "null aggregate");
  return jp::aguard([&] {
    a->p.fetch_groups(stream);
    if (groups) *groups = a->p.groups;
    if (out_j) *out_j = a->p.out_j;
  });
}

jp_status jp_agg_materialize(jp_agg* a, int64_t first, int64_t max_groups, int32_t* out_x, int32_t* out_z,
                             int64_t* out_count, int64_t* out_sum, int64_t* n_written, hipStream_t stream) {
  if (!a || !n_written) return jp::afail(JP_EINVAL, "null aggregate or n_written");
  if (first < 0 || max_groups < 0) return jp::afail(JP_EINVAL, "negative first or max_groups");
  if (max_groups > 0 && (!out_x || !out_z || !out_count || !out_sum))
    return jp::afail(JP_EINVAL, "null output with max_groups > 0");
  *n_written = 0;
  return jp::aguard(
      [&] { *n_written = a->p.materialize(first, max_groups, out_x, out_z, out_count, out_sum, stream); });
}

void jp_agg_destroy(jp_agg* a) {
  if (!a) return;
  (void)hipStreamSynchronize(a->p.stream);
  delete a;
}

}  // extern "C"
