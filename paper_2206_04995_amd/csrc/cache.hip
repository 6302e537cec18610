// Partial result caching (paper Sec. 3).  The result of a Join-Project splits
// by z (the intersection-free partition), so the results of a subset Z_cached
// of the z values can be kept and reused: a later run on the same tables omits
// the S tuples whose z is cached, and its result together with the cached
// pairs is the full result (the two parts are disjoint).
//
// The z values to cache are ranked by CacheScore(z) = cost(z) / space(z):
// * cost(z), the work z brings to the count pass: OUT_{J,z} (join rows
//   reaching z, each an accumulator update in SparseBMM) if z is sparse, and
//   the ratio c_de / c_sp times |X| (one decision per x row) if z is dense -
//   the cost model of the partition (Sec. 2.6);
// * space(z) = 2 + min(k, |X| - k) words, k the number of x with (x, z) in
//   the result: the x list, or its complement in X when k > |X| / 2.
// z values are taken in score order while their space fits the budget.
//
// The cache keeps, per cached z, the x values of its pairs or of their
// complement, and the x values of X (to expand complements).  Its pairs come
// out sorted by (z, x).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/jp.h"
#include "common.h"
#include "plan_impl.h"
#include "pool.h"
#include "prim.h"
#include "stages.h"

struct jp_cache {
  jp::Budget B;
  jp::Arena A{&B};
  int64_t n_r = 0, n_s = 0;  // sizes of the tables the cache was built from
  int64_t NX = 0;             // |X| of the building plan
  int32_t* vals_x = nullptr;  // its x values, ascending
  // cached z (ascending values), per z: complement flag, stored list range, pair count
  int64_t nzc = 0, stored = 0, pairs = 0;
  int32_t* zc_vals = nullptr;     // device, nzc
  std::vector<int32_t> h_zc;      // host copy of zc_vals
  std::vector<int32_t> h_comp;    // 1: the list is the complement in X
  std::vector<int64_t> h_loff;    // list offsets, nzc + 1
  std::vector<int64_t> h_poff;    // pair offsets, nzc + 1
  int32_t* lists = nullptr;       // device: the lists back to back (x values, ascending)
  int64_t *d_poff = nullptr, *d_loff = nullptr;  // device copies of h_poff, h_loff
  int32_t* d_comp = nullptr;                      // device copy of h_comp
};

namespace jp {
namespace {

constexpr int NT = 256;

inline int grid(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 1 << 20))); }

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

__device__ __forceinline__ int64_t find_sorted(const int32_t* __restrict__ a, int64_t n, int32_t v) {
  const int64_t p = lower_bound_dev<int32_t>(a, 0, n, v);
  return (p < n && a[p] == v) ? p : -1;
}

// OUT_{J,z} per z id: every S entry (row y) adds d_R(y) to its z
__global__ void k_outj_z(const int32_t* __restrict__ Ey, const int32_t* __restrict__ scol, int64_t ns,
                         const int32_t* __restrict__ dR, unsigned long long* __restrict__ outjz) {
  GRID_STRIDE(p, ns) {
    const int32_t y = Ey[p + 1] - 1;
    const int32_t d = dR[y];
    if (d) atomicAdd(&outjz[scol[p]], (unsigned long long)d);
  }
}

// k per z id from a chunk of result pairs (z given by value)
__global__ void k_count_z(const int32_t* __restrict__ z, int64_t n, const int32_t* __restrict__ vals_z, int64_t nz,
                          int32_t* __restrict__ kz) {
  GRID_STRIDE(i, n) {
    const int64_t id = find_sorted(vals_z, nz, z[i]);
    if (id >= 0) atomicAdd(&kz[id], 1);
  }
}

// pairs of a chunk whose z is cached (and listed, not complemented): x value at
// the z's cursor; complemented z mark their x id in the z's bitmap row instead
__global__ void k_collect(const int32_t* __restrict__ x, const int32_t* __restrict__ z, int64_t n,
                          const int32_t* __restrict__ zc, int64_t nzc, const int32_t* __restrict__ comp,
                          int32_t* __restrict__ cur, int32_t* __restrict__ lists, const int32_t* __restrict__ vals_x,
                          int64_t nx, const int64_t* __restrict__ brow, uint32_t* __restrict__ bits) {
  GRID_STRIDE(i, n) {
    const int64_t c = find_sorted(zc, nzc, z[i]);
    if (c < 0) continue;
    if (comp[c]) {
      const int64_t xid = find_sorted(vals_x, nx, x[i]);
      atomicOr(&bits[brow[c] + (xid >> 5)], 1u << (xid & 31));
    } else {
      lists[atomicAdd(&cur[c], 1)] = x[i];
    }
  }
}

// complement of one bitmap row: the x values whose bit is clear, ascending (one block)
__global__ void __launch_bounds__(NT) k_complement(const uint32_t* __restrict__ bits, const int32_t* __restrict__ vals_x,
                                                   int64_t nx, int32_t* __restrict__ out) {
  __shared__ int scan_lds[NT / 64];
  __shared__ int64_t base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  for (int64_t x0 = 0; x0 < nx; x0 += NT) {
    const int64_t xi = x0 + threadIdx.x;
    const int miss = (xi < nx && !((bits[xi >> 5] >> (xi & 31)) & 1u)) ? 1 : 0;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    const int incl = wave_incl_scan(miss);
    if (lane == 63) scan_lds[wid] = incl;
    __syncthreads();
    int pre = 0, tot = 0;
    for (int q = 0; q < NT / 64; ++q) {
      if (q < wid) pre += scan_lds[q];
      tot += scan_lds[q];
    }
    if (miss) out[base + pre + incl - miss] = vals_x[xi];
    __syncthreads();
    if (threadIdx.x == 0) base += tot;
    __syncthreads();
  }
}

// S tuples whose z is not cached
__global__ void k_not_cached(const int32_t* __restrict__ sz, int64_t n, const int32_t* __restrict__ zc, int64_t nzc,
                             int32_t* __restrict__ keep) {
  GRID_STRIDE(i, n) { keep[i] = find_sorted(zc, nzc, sz[i]) < 0 ? 1 : 0; }
}

__global__ void k_compact2(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                           const int32_t* __restrict__ keep, const int32_t* __restrict__ E, int64_t n,
                           int32_t* __restrict__ oa, int32_t* __restrict__ ob) {
  GRID_STRIDE(i, n) {
    if (keep[i]) {
      oa[E[i]] = a[i];
      ob[E[i]] = b[i];
    }
  }
}

// first index of a[0, n) with a[i] > v (a ascending)
__device__ __forceinline__ int64_t upper_bound_dev(const int32_t* __restrict__ a, int64_t n, int32_t v) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t m = (lo + hi) >> 1;
    if (a[m] <= v) lo = m + 1;
    else hi = m;
  }
  return lo;
}

// cached pairs [p0, p0 + n) in (z, x) order: pair p belongs to the cached z c
// with poff[c] <= p < poff[c + 1]; its x is the (p - poff[c])-th value of z's
// list, or, for a complemented z, of X minus the list
__global__ void k_expand(const int64_t* __restrict__ poff, const int64_t* __restrict__ loff,
                         const int32_t* __restrict__ comp, const int32_t* __restrict__ zc, int64_t nzc,
                         const int32_t* __restrict__ lists, const int32_t* __restrict__ vals_x, int64_t nx, int64_t p0,
                         int64_t n, int32_t* __restrict__ ox, int32_t* __restrict__ oz) {
  GRID_STRIDE(i, n) {
    const int64_t p = p0 + i;
    int64_t lo = 0, hi = nzc - 1;  // last c with poff[c] <= p
    while (lo < hi) {
      const int64_t m = (lo + hi + 1) >> 1;
      if (poff[m] <= p) lo = m;
      else hi = m - 1;
    }
    const int64_t c = lo, j = p - poff[c];
    const int32_t* list = lists + loff[c];
    const int64_t len = loff[c + 1] - loff[c];
    int32_t x;
    if (!comp[c]) {
      x = list[j];
    } else {
      // smallest q with (q + 1) - (list entries <= X[q]) >= j + 1: the j-th x of X not in the list
      int64_t a = j, b = j + len < nx - 1 ? j + len : nx - 1;
      while (a < b) {
        const int64_t m = (a + b) >> 1;
        if (m + 1 - upper_bound_dev(list, len, vals_x[m]) >= j + 1) b = m;
        else a = m + 1;
      }
      x = vals_x[a];
    }
    ox[i] = x;
    oz[i] = zc[c];
  }
}

// sorted keys (value - INT32_MIN) back to values
__global__ void k_unkey(const uint32_t* __restrict__ k, int64_t n, int32_t* __restrict__ out) {
  GRID_STRIDE(i, n) { out[i] = int32_t(k[i] ^ 0x80000000u); }
}

void lc() { JP_LAUNCH_CHECK(); }

jp_status cfail(int st, const std::string& m) {
  set_last_error(m);
  return jp_status(st);
}

template <class F>
jp_status cguard(F&& f) {
  try {
    f();
    return JP_OK;
  } catch (const Error& e) {
    return cfail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return cfail(JP_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return cfail(JP_EHIP, e.what());
  }
}

void build_cache(jp_cache* c, Plan& p, int64_t budget_bytes, hipStream_t s) {
  p.fetch_totals(s);
  const int64_t total = p.h_tot[0];
  const int64_t NZ = p.NZ, NX = p.NX;
  c->n_r = p.NR;
  c->n_s = p.NS;
  c->NX = NX;
  Arena T(&c->B);
  // cost(z): OUT_{J,z} for sparse z, c_de / c_sp * |X| for dense z
  unsigned long long* outjz = T.alloc<unsigned long long>(std::max<int64_t>(NZ, 1), s);
  fill_i64(reinterpret_cast<int64_t*>(outjz), NZ, 0, s);
  if (p.NS) hipLaunchKernelGGL(k_outj_z, dim3(grid(p.NS)), dim3(NT), 0, s, p.Ey, p.scol, p.NS, p.dR, outjz);
  lc();
  // k(z): pairs per z, from the result in chunks
  int32_t* kz = T.alloc<int32_t>(std::max<int64_t>(NZ, 1), s);
  fill_i32(kz, NZ, 0, s);
  const int64_t chunk = std::min<int64_t>(std::max<int64_t>(total, 1), int64_t(1) << 26);
  int32_t* bx = T.alloc<int32_t>(chunk, s);
  int32_t* bz = T.alloc<int32_t>(chunk, s);
  for (int64_t first = 0; first < total;) {
    const int64_t n = p.materialize(0, JP_PART_ALL, first, chunk, bx, bz, s);
    hipLaunchKernelGGL(k_count_z, dim3(grid(n)), dim3(NT), 0, s, bz, n, p.vals_z, NZ, kz);
    lc();
    first += n;
  }
  std::vector<unsigned long long> h_outjz(size_t(std::max<int64_t>(NZ, 1)));
  std::vector<int32_t> h_kz(size_t(std::max<int64_t>(NZ, 1))), h_flag(size_t(std::max<int64_t>(NZ, 1))),
      h_zv(size_t(std::max<int64_t>(NZ, 1)));
  if (NZ) {
    JP_HIP(hipMemcpyAsync(h_outjz.data(), outjz, NZ * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    JP_HIP(hipMemcpyAsync(h_kz.data(), kz, NZ * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JP_HIP(hipMemcpyAsync(h_flag.data(), p.zflag, NZ * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    JP_HIP(hipMemcpyAsync(h_zv.data(), p.vals_z, NZ * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  }
  JP_HIP(hipStreamSynchronize(s));
  const char* ce = std::getenv("JP_COST_DE_OVER_SP");
  const double c_de = p.h_rec.size() && p.h_rec[0].valid ? p.h_rec[0].ratio : (ce ? std::atof(ce) : 0.05);
  // CacheScore = cost / space; z in score order while their space fits the budget
  std::vector<int64_t> order;
  order.reserve(size_t(NZ));
  std::vector<double> score(size_t(std::max<int64_t>(NZ, 1)));
  std::vector<int64_t> space(size_t(std::max<int64_t>(NZ, 1)));
  for (int64_t z = 0; z < NZ; ++z) {
    const int64_t k = h_kz[size_t(z)];
    if (k == 0) continue;
    space[size_t(z)] = 2 + std::min<int64_t>(k, NX - k);
    const double cost = h_flag[size_t(z)] ? c_de * double(NX) : double(h_outjz[size_t(z)]);
    score[size_t(z)] = cost / double(space[size_t(z)]);
    order.push_back(z);
  }
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return score[size_t(a)] > score[size_t(b)]; });
  std::vector<int64_t> pick;
  int64_t used = 0;
  for (int64_t z : order) {
    const int64_t bytes = 4 * space[size_t(z)];
    if (used + bytes > budget_bytes) continue;
    used += bytes;
    pick.push_back(z);
  }
  std::sort(pick.begin(), pick.end());  // ids ascend with values
  c->nzc = int64_t(pick.size());
  c->h_zc.resize(pick.size());
  c->h_comp.resize(pick.size());
  c->h_loff.assign(pick.size() + 1, 0);
  c->h_poff.assign(pick.size() + 1, 0);
  std::vector<int64_t> h_brow(pick.size(), 0);
  int64_t nbits = 0;
  for (size_t i = 0; i < pick.size(); ++i) {
    const int64_t z = pick[i], k = h_kz[size_t(z)];
    c->h_zc[i] = h_zv[size_t(z)];
    c->h_comp[i] = k > NX - k ? 1 : 0;
    c->h_loff[i + 1] = c->h_loff[i] + (c->h_comp[i] ? NX - k : k);
    c->h_poff[i + 1] = c->h_poff[i] + k;
    h_brow[i] = nbits;
    if (c->h_comp[i]) nbits += (NX + 31) / 32;
  }
  c->stored = c->h_loff.back();
  c->pairs = c->h_poff.back();
  c->vals_x = c->A.alloc<int32_t>(std::max<int64_t>(NX, 1), s);
  if (NX) JP_HIP(hipMemcpyAsync(c->vals_x, p.vals_x, NX * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  c->zc_vals = c->A.alloc<int32_t>(std::max<int64_t>(c->nzc, 1), s);
  c->lists = c->A.alloc<int32_t>(std::max<int64_t>(c->stored, 1), s);
  if (c->nzc == 0) {
    JP_HIP(hipStreamSynchronize(s));
    T.release(s);
    return;
  }
  JP_HIP(hipMemcpyAsync(c->zc_vals, c->h_zc.data(), c->nzc * sizeof(int32_t), hipMemcpyHostToDevice, s));
  c->d_comp = c->A.alloc<int32_t>(c->nzc, s);
  int32_t* comp = c->d_comp;
  JP_HIP(hipMemcpyAsync(comp, c->h_comp.data(), c->nzc * sizeof(int32_t), hipMemcpyHostToDevice, s));
  c->d_poff = c->A.alloc<int64_t>(c->nzc + 1, s);
  c->d_loff = c->A.alloc<int64_t>(c->nzc + 1, s);
  JP_HIP(hipMemcpyAsync(c->d_poff, c->h_poff.data(), (c->nzc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  JP_HIP(hipMemcpyAsync(c->d_loff, c->h_loff.data(), (c->nzc + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  int32_t* cur = T.alloc<int32_t>(c->nzc, s);
  std::vector<int32_t> h_cur(size_t(c->nzc));
  for (int64_t i = 0; i < c->nzc; ++i) h_cur[size_t(i)] = int32_t(c->h_loff[size_t(i)]);
  JP_HIP(hipMemcpyAsync(cur, h_cur.data(), c->nzc * sizeof(int32_t), hipMemcpyHostToDevice, s));
  int64_t* brow = T.alloc<int64_t>(c->nzc, s);
  JP_HIP(hipMemcpyAsync(brow, h_brow.data(), c->nzc * sizeof(int64_t), hipMemcpyHostToDevice, s));
  uint32_t* bits = T.alloc<uint32_t>(std::max<int64_t>(nbits, 1), s);
  fill_u32(bits, nbits, 0u, s);
  // the cached pairs, from the result in chunks (x ascends over the chunks, so
  // each list is collected unordered and sorted below)
  for (int64_t first = 0; first < total;) {
    const int64_t n = p.materialize(0, JP_PART_ALL, first, chunk, bx, bz, s);
    hipLaunchKernelGGL(k_collect, dim3(grid(n)), dim3(NT), 0, s, bx, bz, n, c->zc_vals, c->nzc, comp, cur, c->lists,
                       c->vals_x, NX, brow, bits);
    lc();
    first += n;
  }
  // lists ascending: a segmented radix sort of the x values (offset to be unsigned)
  std::vector<int32_t> seg_base(size_t(c->nzc) + 1);
  for (int64_t i = 0; i <= c->nzc; ++i) seg_base[size_t(i)] = int32_t(c->h_loff[size_t(i)]);
  for (int64_t i = 0; i < c->nzc; ++i) {
    if (!c->h_comp[size_t(i)]) continue;
    hipLaunchKernelGGL(k_complement, dim3(1), dim3(NT), 0, s, bits + h_brow[size_t(i)], c->vals_x, NX,
                       c->lists + c->h_loff[size_t(i)]);
    lc();
  }
  {
    // sort every list: keys = value - INT32_MIN (order preserving), one segment per list
    const int64_t n = c->stored;
    uint32_t* k1 = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
    uint32_t* k2 = T.alloc<uint32_t>(std::max<int64_t>(n, 1), s);
    int32_t* d_base = T.alloc<int32_t>(c->nzc + 1, s);
    JP_HIP(hipMemcpyAsync(d_base, seg_base.data(), (c->nzc + 1) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    int64_t* d_koff = T.alloc<int64_t>(c->nzc + 1, s);
    fill_i64(d_koff, c->nzc + 1, 0, s);
    int32_t* mn = T.alloc<int32_t>(c->nzc, s);
    fill_i32(mn, c->nzc, INT32_MIN, s);
    const SortSegments seg{int(c->nzc), d_base, d_koff, seg_base};
    make_keys(c->lists, n, d_base, int(c->nzc), d_koff, mn, k1, nullptr, nullptr, s);
    uint32_t* sorted = k1;
    if (radix_sort_pairs(k1, nullptr, k2, nullptr, n, 32, s, T, &seg)) sorted = k2;
    if (n) hipLaunchKernelGGL(k_unkey, dim3(grid(n)), dim3(NT), 0, s, sorted, n, c->lists);
    lc();
  }
  JP_HIP(hipStreamSynchronize(s));
  T.release(s);
}

}  // namespace
}  // namespace jp

extern "C" {

jp_status jp_cache_build(jp_plan* p, int64_t budget_bytes, hipStream_t stream, jp_cache** out) {
  using jp::cfail;
  if (!out) return cfail(JP_EINVAL, "out is null");
  *out = nullptr;
  if (!p) return cfail(JP_EINVAL, "plan is null");
  if (p->c) return cfail(JP_EINVAL, "the cache is built from a hybrid plan (this plan runs the classical path)");
  if (p->p.n_inst != 1) return cfail(JP_EINVAL, "the cache is built from a single query");
  if (budget_bytes < 0) return cfail(JP_EINVAL, "negative budget");
  if (!p->p.executed) return cfail(JP_ESTATE, "the cache is built from an executed plan");
  jp_cache* c = new (std::nothrow) jp_cache();
  if (!c) return cfail(JP_ENOMEM, "host allocation failed");
  jp_status st = jp::cguard([&] { jp::build_cache(c, p->p, budget_bytes, stream); });
  if (st != JP_OK) {
    (void)hipStreamSynchronize(stream);
    delete c;
    return st;
  }
  *out = c;
  return JP_OK;
}

jp_status jp_cache_info(const jp_cache* c, int64_t* n_z, int64_t* pairs, int64_t* words) {
  if (!c) return jp::cfail(JP_EINVAL, "cache is null");
  if (n_z) *n_z = c->nzc;
  if (pairs) *pairs = c->pairs;
  if (words) *words = c->stored + 2 * c->nzc;
  return JP_OK;
}

jp_status jp_cache_z(const jp_cache* c, int32_t* z_values) {
  if (!c) return jp::cfail(JP_EINVAL, "cache is null");
  if (z_values && c->nzc) std::memcpy(z_values, c->h_zc.data(), size_t(c->nzc) * sizeof(int32_t));
  return JP_OK;
}

jp_status jp_plan_create_cached(const int32_t* r_x, const int32_t* r_y, int64_t n_r, const int32_t* s_z,
                                const int32_t* s_y, int64_t n_s, const jp_cache* c, const jp_options* opt,
                                hipStream_t stream, jp_plan** out) {
  using jp::cfail;
  if (!out) return cfail(JP_EINVAL, "out is null");
  *out = nullptr;
  if (!c) return cfail(JP_EINVAL, "cache is null");
  if (n_r != c->n_r || n_s != c->n_s) return cfail(JP_EINVAL, "the tables differ in size from the cache's");
  if (n_s < 0 || n_s > INT32_MAX || (n_s > 0 && (!s_z || !s_y))) return cfail(JP_EINVAL, "bad S columns");
  if (c->nzc == 0) return jp_plan_create(r_x, r_y, n_r, s_z, s_y, n_s, opt, stream, out);
  jp::Arena T;
  int32_t *fz = nullptr, *fy = nullptr;
  int64_t nf = 0;
  jp_status st = jp::cguard([&] {
    using namespace jp;
    const int64_t NSa = std::max<int64_t>(n_s, 1);
    int32_t* keep = T.alloc<int32_t>(NSa, stream);
    if (n_s) hipLaunchKernelGGL(k_not_cached, dim3(grid(n_s)), dim3(NT), 0, stream, s_z, n_s, c->zc_vals, c->nzc, keep);
    lc();
    int32_t* E = T.alloc<int32_t>(n_s + 1, stream);
    scan_excl_i32(keep, E, n_s, stream, T);
    int32_t h = 0;
    JP_HIP(hipMemcpyAsync(&h, E + n_s, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    JP_HIP(hipStreamSynchronize(stream));
    nf = h;
    fz = T.alloc<int32_t>(std::max<int64_t>(nf, 1), stream);
    fy = T.alloc<int32_t>(std::max<int64_t>(nf, 1), stream);
    if (n_s) hipLaunchKernelGGL(k_compact2, dim3(grid(n_s)), dim3(NT), 0, stream, s_z, s_y, keep, E, n_s, fz, fy);
    lc();
  });
  if (st == JP_OK) st = jp_plan_create(r_x, r_y, n_r, fz, fy, nf, opt, stream, out);
  (void)hipStreamSynchronize(stream);  // the plan holds its own copies once its creation work is done
  T.release(stream);
  return st;
}

jp_status jp_cache_materialize(const jp_cache* c, int64_t first, int64_t max_pairs, int32_t* out_x, int32_t* out_z,
                               int64_t* n_written, hipStream_t stream) {
  using jp::cfail;
  if (!c || !n_written) return cfail(JP_EINVAL, "cache or n_written is null");
  if (first < 0 || max_pairs < 0) return cfail(JP_EINVAL, "negative first or max_pairs");
  if (max_pairs > 0 && (!out_x || !out_z)) return cfail(JP_EINVAL, "null output with max_pairs > 0");
  *n_written = 0;
  if (first > c->pairs) return cfail(JP_ERANGE, "first beyond the number of cached pairs");
  const int64_t n = std::min(max_pairs, c->pairs - first);
  if (n <= 0) return JP_OK;
  return jp::cguard([&] {
    using namespace jp;
    hipLaunchKernelGGL(k_expand, dim3(grid(n)), dim3(NT), 0, stream, c->d_poff, c->d_loff, c->d_comp, c->zc_vals,
                       c->nzc, c->lists, c->vals_x, c->NX, first, n, out_x, out_z);
    lc();
    JP_HIP(hipStreamSynchronize(stream));
    *n_written = n;
  });
}

void jp_cache_destroy(jp_cache* c) {
  if (!c) return;
  c->A.release(nullptr);
  delete c;
}

}  // extern "C"
