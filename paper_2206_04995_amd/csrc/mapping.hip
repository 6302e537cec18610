// Mapping of x, y, z values to dense order-preserving ids (paper Sec. 2.2)
// and the CSR builds of R and S (Sec. 2.4).  Ids come from sorted runs of
// equal keys, so id order equals value order; the join key y is mapped from
// S first and R tuples whose y is absent from S are dropped (optimisation 2).
#include "common.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

constexpr int NT = 256;

inline int grid(int64_t n, int cap = 1 << 20) {
  int64_t g = (n + NT - 1) / NT;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

// k_make_keys takes four elements per thread and step (positions i0 +
// u * blockDim.x, u < 4, increasing) and issues their loads before using them:
// one load at a time, consumed at once, would leave each thread waiting on
// memory.  (The same form made the carried-key and direct semi-join kernels
// slower, so they keep one element per step.)
constexpr int UNR = 4;

__device__ __forceinline__ int64_t chunk_end(int64_t n) {
  const int64_t c1 = chunk_first() + JP_CHUNK;
  return c1 < n ? c1 : n;
}

__global__ void k_make_keys(const int32_t* __restrict__ v, int64_t n, const int32_t* __restrict__ ebase,
                            int n_inst, const int64_t* __restrict__ koff, const int32_t* __restrict__ mn,
                            uint32_t* __restrict__ keys, uint32_t* __restrict__ payload,
                            const int32_t* __restrict__ pay_src) {
  SegCursor<int32_t> cur(ebase, n_inst);
  cur.seed(int32_t(chunk_first()));
  const int64_t c1 = chunk_end(n);
  const int64_t step = blockDim.x;
  for (int64_t i0 = chunk_first() + threadIdx.x; i0 < c1; i0 += UNR * step) {
    int32_t vv[UNR], pp[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t i = i0 + u * step;
      vv[u] = i < c1 ? v[i] : 0;
      pp[u] = (pay_src && i < c1) ? pay_src[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t i = i0 + u * step;
      if (i >= c1) break;
      const int inst = cur(int32_t(i));
      keys[i] = uint32_t(koff[inst] + (int64_t(vv[u]) - int64_t(mn[inst])));
      if (payload) payload[i] = pay_src ? uint32_t(pp[u]) : uint32_t(i);
    }
  }
}

// Run ids of sorted keys in two passes over the keys (a head starts a run of
// equal keys): k_run_heads counts the heads of each tile, and k_run_ids ranks
// the heads of its tile (offset by the scanned tile counts) and writes, for
// every head, its position first[id] and its original value
// vals[id] = key - koff[inst] + mn[inst].  A wave owns 64 * RUN_IT consecutive
// keys and takes them 64 at a time, so loads and stores are coalesced and the
// head ranks are ballot bit counts.  Per position it writes, by mode:
//   RUN_E      E[i] = runs started before position i (E[n] = the run count);
//   RUN_NONE   nothing (ids of segment starts come from first[], ids_at_bases);
//   RUN_CARRY  the id of position i as payload[i], and the key of the carried
//              value c.v[i] under a second layout (c.koff, c.mn) as c.keys[i],
//              ready for the next sort.
constexpr int RUN_NT = 256;
constexpr int RUN_IT = 8;
constexpr int RUN_TILE = RUN_NT * RUN_IT;
constexpr int RUN_WAVES = RUN_NT / 64;
constexpr int RUN_WTILE = 64 * RUN_IT;
enum RunMode { RUN_E = 0, RUN_NONE = 1, RUN_CARRY = 2 };

__device__ __forceinline__ uint64_t run_head_bits(const uint32_t* __restrict__ keys, int64_t n, int64_t w0,
                                                  const uint32_t (&k)[RUN_IT], uint64_t (&hb)[RUN_IT]) {
  const int lane = lane_id();
  uint32_t before = (w0 > 0 && w0 - 1 < n) ? keys[w0 - 1] : 0u;  // key in front of the wave's first
  uint64_t cnt = 0;
#pragma unroll
  for (int j = 0; j < RUN_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    uint32_t prev = __shfl_up(k[j], 1, 64);
    if (lane == 0) prev = before;
    const bool head = i < n && (i == 0 || prev != k[j]);
    hb[j] = ballot(head);
    cnt += uint64_t(__popcll(hb[j]));
    before = __builtin_amdgcn_readlane(k[j], 63);
  }
  return cnt;
}

__global__ void __launch_bounds__(RUN_NT) k_run_heads(const uint32_t* __restrict__ keys, int64_t n,
                                                      int32_t* __restrict__ sums) {
  __shared__ int32_t part[RUN_WAVES];
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int64_t w0 = int64_t(blockIdx.x) * RUN_TILE + int64_t(wid) * RUN_WTILE;
  uint32_t k[RUN_IT];
  uint64_t hb[RUN_IT];
#pragma unroll
  for (int j = 0; j < RUN_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    k[j] = i < n ? keys[i] : 0u;
  }
  const int c = int(run_head_bits(keys, n, w0, k, hb));
  if (lane == 0) part[wid] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
#pragma unroll
    for (int w = 0; w < RUN_WAVES; ++w) t += part[w];
    sums[blockIdx.x] = t;
  }
}


template <int MODE>
__global__ void __launch_bounds__(RUN_NT) k_run_ids(const uint32_t* __restrict__ keys, int64_t n,
                                                    const int32_t* __restrict__ offs, const int64_t* __restrict__ koff,
                                                    const int32_t* __restrict__ mn, int n_inst, int32_t* __restrict__ E,
                                                    int32_t* __restrict__ first, int32_t* __restrict__ vals,
                                                    int32_t* __restrict__ total, RunCarry c,
                                                    int32_t* __restrict__ table) {
  __shared__ int32_t part[RUN_WAVES];
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int64_t w0 = int64_t(blockIdx.x) * RUN_TILE + int64_t(wid) * RUN_WTILE;
  const uint64_t ltm = lanemask_lt();
  uint32_t k[RUN_IT];
  int32_t cv[RUN_IT];
  uint64_t hb[RUN_IT];
#pragma unroll
  for (int j = 0; j < RUN_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    k[j] = i < n ? keys[i] : 0u;
    if (MODE == RUN_CARRY) cv[j] = i < n ? c.v[i] : 0;
  }
  const int cnt = int(run_head_bits(keys, n, w0, k, hb));
  if (lane == 0) part[wid] = cnt;
  __syncthreads();
  int run = offs ? offs[blockIdx.x] : 0, btot = 0;
#pragma unroll
  for (int w = 0; w < RUN_WAVES; ++w) {
    if (w < wid) run += part[w];
    btot += part[w];
  }
  SegCursor<int64_t> kcur(koff, n_inst);
  if (w0 < n) kcur.seed(int64_t(__builtin_amdgcn_readlane(k[0], 0)));  // the wave's smallest key
#pragma unroll
  for (int j = 0; j < RUN_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    const int h = int((hb[j] >> lane) & 1u);
    const int r = run + __popcll(hb[j] & ltm);  // runs started before i
    if (i < n) {
      if (MODE == RUN_E) E[i] = r;
      if (h || MODE == RUN_CARRY) {
        const int inst = kcur(int64_t(k[j]));
        if (h) {
          first[r] = int32_t(i);
          vals[r] = int32_t(int64_t(k[j]) - koff[inst] + int64_t(mn[inst]));
          if (table) table[k[j]] = r;
        }
        if (MODE == RUN_CARRY) {
          c.keys[i] = uint32_t(c.koff[inst] + (int64_t(cv[j]) - int64_t(c.mn[inst])));
          c.payload[i] = uint32_t(r + h - 1);
        }
      }
    }
    run += __popcll(hb[j]);
  }
  // the grid's last block holds the total: E[n], first[total] = n
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    const int t = (offs ? offs[blockIdx.x] : 0) + btot;
    if (MODE == RUN_E) E[n] = t;
    first[t] = int32_t(n);
    if (total) *total = t;
  }
}

// out[i] = runs started before ebase[i] = lower bound of ebase[i] in first[0, *total)
__global__ void k_ids_at_bases(const int32_t* __restrict__ first, const int32_t* __restrict__ total,
                               const int32_t* __restrict__ ebase, int n_inst, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n_inst) return;
  const int32_t p = ebase[i];
  int64_t lo = 0, hi = *total;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (first[mid] < p) lo = mid + 1;
    else hi = mid;
  }
  out[i] = int32_t(lo);
}

__global__ void k_gather_bases(const int32_t* __restrict__ E, const int32_t* __restrict__ ebase, int n_inst,
                               int32_t* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_inst) out[i] = E[ebase[i]];
}

__global__ void k_semijoin(const int32_t* __restrict__ ry, int64_t n, const int32_t* __restrict__ ebase, int n_inst,
                           const int32_t* __restrict__ vals_y, const int32_t* __restrict__ y_base,
                           int32_t* __restrict__ keep, int32_t* __restrict__ yid) {
  SegCursor<int32_t> cur(ebase, n_inst);
  cur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(g, n, JP_CHUNK) {
    const int inst = cur(int32_t(g));
    int32_t v = ry[g];
    int64_t lo = y_base[inst], hi = y_base[inst + 1];
    int64_t pos = lower_bound_dev<int32_t>(vals_y, lo, hi, v);
    bool ok = pos < hi && vals_y[pos] == v;
    keep[g] = ok ? 1 : 0;
    yid[g] = ok ? int32_t(pos) : -1;
  }
}

// direct-address table of the y keys (used when the key space is small, as
// for naturally dense domains): table[key] = id, one thread per run of the
// y-sorted keys (first[id] is the run's first position)
__global__ void k_fill_direct(const uint32_t* __restrict__ keys, const int32_t* __restrict__ first,
                              const int32_t* __restrict__ total, int32_t* __restrict__ table) {
  const int64_t runs = *total;
  GRID_STRIDE(r, runs) table[keys[first[r]]] = int32_t(r);
}

__global__ void k_semijoin_direct(const int32_t* __restrict__ ry, int64_t n, const int32_t* __restrict__ ebase,
                                  int n_inst, const int64_t* __restrict__ koff, const int32_t* __restrict__ mn,
                                  const int32_t* __restrict__ table, int32_t* __restrict__ keep,
                                  int32_t* __restrict__ yid) {
  SegCursor<int32_t> cur(ebase, n_inst);
  cur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(g, n, JP_CHUNK) {
    const int inst = cur(int32_t(g));
    const int64_t rel = int64_t(ry[g]) - int64_t(mn[inst]);
    const int64_t range = koff[inst + 1] - koff[inst];
    const int32_t id = (rel >= 0 && rel < range) ? table[koff[inst] + rel] : -1;
    keep[g] = id >= 0 ? 1 : 0;
    yid[g] = id;
  }
}

// Semi-join, compaction and x keys in one pass (Sec. 2.2, optimisation 2):
// per R tuple its y id (direct table or binary search among the instance's y
// values), and for the kept tuples, in order, the key of x under the layout
// (koff_x, xmin) and the y id.  A tile places its kept tuples at the
// look-back prefix of the kept counts (lookback_exclusive), and writes
// rpbase[i] = kept tuples before ebase[i] for the instances starting in it.
constexpr int SJ_NT = 512;  // 8192-tuple tiles (faster with one buffer per instance)
constexpr int SJ_IT = 16;
constexpr int SJ_WTILE = 64 * SJ_IT;
constexpr int SJ_TILE = SJ_NT * SJ_IT;

template <bool DIRECT>
__global__ void __launch_bounds__(SJ_NT) k_semijoin_compact(SemiJoinIn in, uint32_t* __restrict__ xk,
                                                            uint32_t* __restrict__ oy, int32_t* __restrict__ rpbase,
                                                            int32_t* __restrict__ total, uint64_t* __restrict__ status,
                                                            int64_t ntiles) {
  __shared__ int64_t s_tile;
  __shared__ int32_t s_wsum[SJ_NT / 64];
  __shared__ int64_t s_excl;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t ltm = lanemask_lt();
  if (threadIdx.x == 0) s_tile = lookback_ticket(status, ntiles);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t w0 = tile * SJ_TILE + int64_t(wid) * SJ_WTILE;
  const int64_t wend = w0 + SJ_WTILE < in.n ? w0 + SJ_WTILE : in.n;
  int32_t xr[SJ_IT], yr[SJ_IT];
  uint32_t xv[SJ_IT];
  int32_t yid[SJ_IT];
  uint32_t starts = 0;  // bit j: this lane's position of row j starts an instance
  int cnt = 0;
  // the instance of the wave's first position (wave-uniform)
  const int i0 = DIRECT && w0 < in.n ? wave_find_inst<int32_t>(in.ebase, in.n_inst, int32_t(w0)) : 0;
  if (DIRECT && w0 < in.n && int64_t(in.ebase[i0 + 1]) >= wend) {
    // the wave's positions lie in one instance (all but the waves at instance
    // bounds): its layout constants are wave-uniform, and every load (columns,
    // then the y lookups) is issued before any is used
    const int64_t k0 = in.koff_y[i0], range = in.koff_y[i0 + 1] - k0;
    const int64_t ymn = in.ymin[i0], xoff = in.koff_x[i0] - int64_t(in.xmin[i0]);
    const int64_t st = in.ebase[i0];
    // element i at px[i - st] (the instance's own buffers, or the concatenation)
    const int32_t* px = in.cx ? in.cx[i0] : in.rx + st;
    const int32_t* py = in.cy ? in.cy[i0] : in.ry + st;
#pragma unroll
    for (int j = 0; j < SJ_IT; ++j) {
      const int64_t i = w0 + j * 64 + lane;
      const int64_t ic = i < wend ? i : wend - 1;
      xr[j] = px[ic - st];
      yr[j] = py[ic - st];
      if (i == st) starts |= 1u << j;
    }
    int32_t t[SJ_IT];
#pragma unroll
    for (int j = 0; j < SJ_IT; ++j) {
      const int64_t rel = int64_t(yr[j]) - ymn;
      t[j] = in.table[rel >= 0 && rel < range ? k0 + rel : 0];
    }
#pragma unroll
    for (int j = 0; j < SJ_IT; ++j) {
      const int64_t rel = int64_t(yr[j]) - ymn;
      const bool ok = rel >= 0 && rel < range && w0 + j * 64 + lane < wend;
      yid[j] = ok ? t[j] : -1;
      xv[j] = uint32_t(xoff + int64_t(xr[j]));
      cnt += __popcll(ballot(yid[j] >= 0));
    }
  } else {
    SegCursor<int32_t> cur(in.ebase, in.n_inst);
    if (w0 < in.n) cur.seed(int32_t(w0));
    // columns and instances of all rows first (loads at clamped, valid indices), then the y lookups
    int32_t ins[SJ_IT];
#pragma unroll
    for (int j = 0; j < SJ_IT; ++j) {
      const int64_t i = w0 + j * 64 + lane;
      const int64_t ic = i < in.n ? i : in.n - 1;
      ins[j] = 0;
      if (in.cx) {
        // per-instance buffers: the instance first (the clamped position's, for lanes past the end)
        const int k = cur(int32_t(ic));
        xr[j] = in.cx[k][ic - cur.lo];
        yr[j] = in.cy[k][ic - cur.lo];
        if (i < in.n) {
          ins[j] = k;
          if (i == cur.lo) starts |= 1u << j;
        }
      } else {
        xr[j] = in.rx[ic];
        yr[j] = in.ry[ic];
        if (i < in.n) {
          ins[j] = cur(int32_t(i));
          if (i == cur.lo) starts |= 1u << j;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < SJ_IT; ++j) {
      const int inst = ins[j];
      int32_t id = -1;
      if (DIRECT) {
        const int64_t rel = int64_t(yr[j]) - int64_t(in.ymin[inst]);
        const int64_t k0 = in.koff_y[inst];
        const bool ok = rel >= 0 && rel < in.koff_y[inst + 1] - k0;
        const int32_t t = in.table[ok ? k0 + rel : 0];
        id = ok ? t : -1;
      } else {
        const int64_t lo = in.y_base[inst], hi = in.y_base[inst + 1];
        const int64_t pos = lower_bound_dev<int32_t>(in.vals_y, lo, hi, yr[j]);
        if (pos < hi && in.vals_y[pos] == yr[j]) id = int32_t(pos);
      }
      yid[j] = w0 + j * 64 + lane < in.n ? id : -1;
      xv[j] = uint32_t(in.koff_x[inst] + (int64_t(xr[j]) - int64_t(in.xmin[inst])));
      cnt += __popcll(ballot(yid[j] >= 0));
    }
  }
  if (lane == 0) s_wsum[wid] = cnt;
  __syncthreads();
  int32_t woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < SJ_NT / 64; ++w) {
    if (w < wid) woff += s_wsum[w];
    btot += s_wsum[w];
  }
  if (wid == 0) {
    const int64_t excl = lookback_exclusive(status, tile, ntiles, btot);
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  int64_t run = s_excl + woff;  // wave-uniform
#pragma unroll
  for (int j = 0; j < SJ_IT; ++j) {
    const uint64_t b = ballot(yid[j] >= 0);
    const int64_t before = run + __popcll(b & ltm);
    if (yid[j] >= 0) {
      xk[before] = xv[j];
      oy[before] = uint32_t(yid[j]);
    }
    if ((starts >> j) & 1u) {
      // the instance holding this position and any empty ones starting here
      const int32_t i = int32_t(w0 + j * 64 + lane);
      for (int k = find_inst<int32_t>(in.ebase, in.n_inst, i); k >= 0 && in.ebase[k] == i; --k)
        rpbase[k] = int32_t(before);
    }
    run += __popcll(b);
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) {
    const int32_t t = int32_t(s_excl + btot);
    *total = t;
    for (int k = in.n_inst; k >= 0 && in.ebase[k] == in.n; --k) rpbase[k] = t;
  }
}

__global__ void k_run_lengths(const int32_t* __restrict__ first, int64_t n_id, int32_t* __restrict__ m) {
  GRID_STRIDE(i, n_id) { m[i] = first[i + 1] - first[i]; }
}

// Histogram with per-block aggregation in an LDS hash table, so frequent keys
// (skewed join keys) cost one global atomic per block instead of one per
// element; keys that do not find a slot go straight to global memory.
constexpr int HG_SLOTS = 4096;
constexpr int HG_PER_BLOCK = 1 << 14;

__global__ void __launch_bounds__(NT) k_histogram(const uint32_t* __restrict__ v, int64_t n, int32_t* __restrict__ h) {
  __shared__ uint32_t key[HG_SLOTS];
  __shared__ int32_t cnt[HG_SLOTS];
  for (int i = threadIdx.x; i < HG_SLOTS; i += NT) {
    key[i] = 0xFFFFFFFFu;
    cnt[i] = 0;
  }
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * HG_PER_BLOCK;
  const int64_t b1 = b0 + HG_PER_BLOCK < n ? b0 + HG_PER_BLOCK : n;
  // eight values' loads in flight (clamped indices), then their table updates
  constexpr int HG_U = 8;
  for (int64_t i0 = b0 + threadIdx.x; i0 < b1; i0 += HG_U * NT) {
    uint32_t kk[HG_U];
#pragma unroll
    for (int u = 0; u < HG_U; ++u) {
      const int64_t i = i0 + u * NT;
      kk[u] = v[i < b1 ? i : b1 - 1];
    }
#pragma unroll
    for (int u = 0; u < HG_U; ++u) {
      if (i0 + u * NT >= b1) break;
      const uint32_t k = kk[u];
      uint32_t s = (k * 0x9E3779B1u) >> 20;  // 12-bit slot
      bool done = false;
      for (int probe = 0; probe < 2 && !done; ++probe) {
        uint32_t old = atomicCAS(&key[s], 0xFFFFFFFFu, k);
        if (old == 0xFFFFFFFFu || old == k) {
          atomicAdd(&cnt[s], 1);
          done = true;
        } else {
          s = (s + 1) & (HG_SLOTS - 1);
        }
      }
      if (!done) atomicAdd(&h[k], 1);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < HG_SLOTS; i += NT)
    if (cnt[i]) atomicAdd(&h[key[i]], cnt[i]);
}

// Histogram over a small key space (at most SMALL_BINS keys): every block bins
// a long run of elements in LDS and adds its non-zero bins to the global counts
// (the hash aggregation above sends most elements of a space wider than its
// 4096 slots to global atomics, many of them on the same few thousand keys).
constexpr int SMALL_BINS = 16384;

__global__ void __launch_bounds__(NT) k_histogram_small(const uint32_t* __restrict__ v, int64_t n, int nbins,
                                                        int64_t per_block, int32_t* __restrict__ h) {
  __shared__ int32_t bins[SMALL_BINS];
  for (int i = threadIdx.x; i < nbins; i += NT) bins[i] = 0;
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * per_block;
  const int64_t b1 = b0 + per_block < n ? b0 + per_block : n;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) atomicAdd(&bins[v[i]], 1);
  __syncthreads();
  for (int i = threadIdx.x; i < nbins; i += NT)
    if (bins[i]) atomicAdd(&h[i], bins[i]);
}

__global__ void k_out_j(const int32_t* __restrict__ dR, const int32_t* __restrict__ dS, int64_t n_y,
                        const int32_t* __restrict__ y_base, int n_inst, int64_t* __restrict__ out_j) {
  if (n_inst == 1) {  // grid-stride sum, one atomic per block
    __shared__ int64_t s_part[NT / 64];
    int64_t acc = 0;
    for (int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; y < n_y; y += int64_t(gridDim.x) * blockDim.x)
      acc += int64_t(dR[y]) * int64_t(dS[y]);
    acc = wave_sum(acc);
    if (lane_id() == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t t = 0;
      for (int w = 0; w < NT / 64; ++w) t += s_part[w];
      if (t) atomicAdd((unsigned long long*)&out_j[0], (unsigned long long)t);
    }
    return;
  }
  // a block per chunk of JP_CHUNK keys, walked in wave-uniform steps with an instance cursor
  SegCursor<int32_t> ycur(y_base, n_inst);
  ycur.seed(int32_t(chunk_first()));
  const int64_t c1 = chunk_first() + JP_CHUNK < n_y ? chunk_first() + JP_CHUNK : n_y;
  for (int64_t b = chunk_first() + (threadIdx.x & ~63); b < c1; b += blockDim.x) {
    const int64_t y = b + lane_id();
    int64_t prod = 0;
    int inst = 0;
    if (y < c1) {
      prod = int64_t(dR[y]) * int64_t(dS[y]);
      inst = ycur(int32_t(y));
    }
    const int i0 = __shfl(inst, 0, 64);
    if (ballot(y < c1 && inst != i0) == 0) {
      const int64_t s = wave_sum(prod);
      if (lane_id() == 0 && s) atomicAdd((unsigned long long*)&out_j[i0], (unsigned long long)s);
    } else if (prod) {
      atomicAdd((unsigned long long*)&out_j[inst], (unsigned long long)prod);
    }
  }
}


// ------------------------------------------------- direct-range mapping
// When the values of a column fill their range densely (the key space, the sum
// of the instances' value ranges, is within a small multiple of the column
// length), ids need no sort (Sec. 2.2, optimisation 1: columns that already
// hold natural numbers skip the dictionary).  A key histogram over the key
// space gives each value's count; the exclusive scan of the presence flags
// gives the order-preserving id of every present key, the same ids a sort
// assigns; the exclusive scan of the counts gives each key's first position in
// key order, and a scatter with one atomic cursor per key places the elements
// there (order inside a key is arbitrary).

// h[key(i)] += 1 for elements whose filter entry is >= 0 (all if filter is
// null), aggregated per block in an LDS hash table like k_histogram
__global__ void __launch_bounds__(NT) k_key_hist(const int32_t* __restrict__ v, int64_t n,
                                                 const int32_t* __restrict__ ebase, int n_inst,
                                                 const int64_t* __restrict__ koff, const int32_t* __restrict__ mn,
                                                 const int32_t* __restrict__ filter, int32_t* __restrict__ h) {
  __shared__ uint32_t key[HG_SLOTS];
  __shared__ int32_t cnt[HG_SLOTS];
  for (int i = threadIdx.x; i < HG_SLOTS; i += NT) {
    key[i] = 0xFFFFFFFFu;
    cnt[i] = 0;
  }
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * HG_PER_BLOCK;
  const int64_t b1 = b0 + HG_PER_BLOCK < n ? b0 + HG_PER_BLOCK : n;
  SegCursor<int32_t> cur(ebase, n_inst);
  cur.seed(int32_t(b0 < n ? b0 : 0));
  for (int64_t i = b0 + threadIdx.x; i < b1; i += NT) {
    if (filter && filter[i] < 0) continue;
    const int inst = cur(int32_t(i));
    const uint32_t k = uint32_t(koff[inst] + (int64_t(v[i]) - int64_t(mn[inst])));
    uint32_t s = (k * 0x9E3779B1u) >> 20;  // 12-bit slot
    bool done = false;
    for (int probe = 0; probe < 2 && !done; ++probe) {
      uint32_t old = atomicCAS(&key[s], 0xFFFFFFFFu, k);
      if (old == 0xFFFFFFFFu || old == k) {
        atomicAdd(&cnt[s], 1);
        done = true;
      } else {
        s = (s + 1) & (HG_SLOTS - 1);
      }
    }
    if (!done) atomicAdd(&h[k], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < HG_SLOTS; i += NT)
    if (cnt[i]) atomicAdd(&h[key[i]], cnt[i]);
}

__global__ void k_presence(const int32_t* __restrict__ cnt, int64_t n_keys, int32_t* __restrict__ pres) {
  GRID_STRIDE(k, n_keys) { pres[k] = cnt[k] > 0 ? 1 : 0; }
}

// for every present key: its id E[key], the id's original value, and
// optionally its count and first position C[key]; first[n_id] = C[n_keys]
__global__ void k_key_ids(const int32_t* __restrict__ cnt, int64_t n_keys, const int32_t* __restrict__ E,
                          const int32_t* __restrict__ C, const int64_t* __restrict__ koff,
                          const int32_t* __restrict__ mn, int n_inst, int32_t* __restrict__ vals,
                          int32_t* __restrict__ m, int32_t* __restrict__ first) {
  SegCursor<int64_t> kc(koff, n_inst);
  GRID_STRIDE(k, n_keys) {
    const int32_t c = cnt[k];
    if (c > 0) {
      const int inst = kc(k);
      const int32_t id = E[k];
      vals[id] = int32_t(k - koff[inst] + int64_t(mn[inst]));
      if (m) m[id] = c;
      if (first) first[id] = C[k];
    }
    if (k == n_keys - 1 && first) first[E[n_keys]] = C[n_keys];
  }
}

// out[i] = E[koff[i]] for i in [0, n_inst]
__global__ void k_bases_from_koff(const int32_t* __restrict__ E, const int64_t* __restrict__ koff, int n_inst,
                                  int32_t* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_inst) out[i] = E[koff[i]];
}

// S placed in z order: position cur[zkey]++ (cur starts as the scan of the z
// counts) receives the y key of the tuple and its z id, ready for the stable
// sort by y that yields the CSR of S by y with ascending z inside each row
__global__ void k_scatter_z(const int32_t* __restrict__ sz, const int32_t* __restrict__ sy, int64_t n,
                            const int32_t* __restrict__ ebase, int n_inst, const int64_t* __restrict__ koff_z,
                            const int32_t* __restrict__ zmin, const int64_t* __restrict__ koff_y,
                            const int32_t* __restrict__ ymin, const int32_t* __restrict__ Ez,
                            int32_t* __restrict__ cur, uint32_t* __restrict__ yk, uint32_t* __restrict__ zid) {
  SegCursor<int32_t> sc(ebase, n_inst);
  sc.seed(int32_t(chunk_first()));
  CHUNK_LOOP(i, n, JP_CHUNK) {
    const int inst = sc(int32_t(i));
    const int32_t zv = sz[i], yv = sy[i];
    const int64_t zk = koff_z[inst] + (int64_t(zv) - int64_t(zmin[inst]));
    const int32_t p = atomicAdd(&cur[zk], 1);
    yk[p] = uint32_t(koff_y[inst] + (int64_t(yv) - int64_t(ymin[inst])));
    zid[p] = uint32_t(Ez[zk]);
  }
}

// R' grouped by x: every kept R tuple (yid >= 0) writes its y id at position
// cur[xkey]++ (cur starts as the scan of the kept x counts)
__global__ void k_scatter_x(const int32_t* __restrict__ rx, const int32_t* __restrict__ yid, int64_t n,
                            const int32_t* __restrict__ ebase, int n_inst, const int64_t* __restrict__ koff_x,
                            const int32_t* __restrict__ xmin, int32_t* __restrict__ cur, int32_t* __restrict__ rcol) {
  SegCursor<int32_t> sc(ebase, n_inst);
  sc.seed(int32_t(chunk_first()));
  CHUNK_LOOP(g, n, JP_CHUNK) {
    const int32_t y = yid[g];
    const int inst = sc(int32_t(g));
    if (y >= 0) {
      const int64_t xk = koff_x[inst] + (int64_t(rx[g]) - int64_t(xmin[inst]));
      rcol[atomicAdd(&cur[xk], 1)] = y;
    }
  }
}

// gather of per-instance device columns into one concatenated buffer; with
// mn/mx non-null also each instance's minimum and maximum (the key layout of
// the mapping), so the column is read once for both
__device__ __forceinline__ void flush_minmax(int inst, int32_t lo, int32_t hi, int32_t* mn, int32_t* mx) {
  // whole wave: one atomic pair when every lane holds the same instance
  const int i0 = __builtin_amdgcn_readfirstlane(inst);
  if (ballot(inst != i0) == 0) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int32_t a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
      lo = a < lo ? a : lo;
      hi = b > hi ? b : hi;
    }
    if (lane_id() == 0 && inst >= 0) {
      atomicMin(&mn[inst], lo);
      atomicMax(&mx[inst], hi);
    }
  } else if (inst >= 0) {
    atomicMin(&mn[inst], lo);
    atomicMax(&mx[inst], hi);
  }
}

__global__ void k_gather_cols(const int32_t* const* __restrict__ src, const int32_t* __restrict__ base, int n_inst,
                              int64_t n, int32_t* __restrict__ dst, int32_t* __restrict__ mn,
                              int32_t* __restrict__ mx) {
  const int64_t c0 = chunk_first();
  const int64_t c1 = c0 + JP_CHUNK < n ? c0 + JP_CHUNK : n;
  const int64_t step = blockDim.x;
  const int i0 = wave_find_inst<int32_t>(base, n_inst, int32_t(c0));
  if (int64_t(base[i0 + 1]) >= c1) {
    // the chunk lies in one instance (all but the chunks at instance bounds): no per-element lookups
    // all of a thread's JP_CHUNK / 256 loads in flight at once (clamped indices, no branches), then the stores
    const int32_t* col = src[i0] + (c0 - base[i0]);
    int32_t lo = INT32_MAX, hi = INT32_MIN;
    constexpr int GU = JP_CHUNK / 256;  // elements per thread (the launch uses 256 threads)
    int32_t vv[GU];
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int64_t g = c0 + threadIdx.x + u * step;
      vv[u] = col[(g < c1 ? g : c1 - 1) - c0];
    }
#pragma unroll
    for (int u = 0; u < GU; ++u) {
      const int64_t g = c0 + threadIdx.x + u * step;
      if (g < c1) {
        if (dst) dst[g] = vv[u];
        lo = vv[u] < lo ? vv[u] : lo;
        hi = vv[u] > hi ? vv[u] : hi;
      }
    }
    if (mn) {
      // the block's min and max (one instance): one atomic pair per block
      __shared__ int32_t s_lo[JP_CHUNK / 64], s_hi[JP_CHUNK / 64];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const int32_t a = __shfl_xor(lo, o, 64), b = __shfl_xor(hi, o, 64);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
      }
      const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
      if (lane_id() == 0) {
        s_lo[wid] = lo;
        s_hi[wid] = hi;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
          lo = s_lo[w] < lo ? s_lo[w] : lo;
          hi = s_hi[w] > hi ? s_hi[w] : hi;
        }
        atomicMin(&mn[i0], lo);
        atomicMax(&mx[i0], hi);
      }
    }
    return;
  }
  SegCursor<int32_t> cur(base, n_inst);
  cur.seed(int32_t(c0));
  const int32_t* col = nullptr;
  int last = -1;                           // instance of `col`
  int acc = -1;                            // instance whose values lo and hi hold
  int32_t lo = INT32_MAX, hi = INT32_MIN;
  // four elements per thread and step: their source addresses first, then the
  // four loads in flight together, then the stores (and the min and max, in
  // element order, so a lane's values move to the next instance's at its bound)
  for (int64_t g0 = chunk_first() + threadIdx.x; g0 < c1; g0 += 4 * step) {
    const int32_t* at[4];
    int iu[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t g = g0 + u * step;
      at[u] = nullptr;
      iu[u] = -1;
      if (g < c1) {
        const int inst = cur(int32_t(g));
        if (inst != last) {
          last = inst;
          col = src[inst];
        }
        at[u] = col + (g - cur.lo);
        iu[u] = inst;
      }
    }
    int32_t vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) vv[u] = at[u] ? *at[u] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (iu[u] >= 0) {
        if (dst) dst[g0 + u * step] = vv[u];
        if (mn) {
          if (iu[u] != acc) {  // rare: at instance bounds
            if (acc >= 0) {
              atomicMin(&mn[acc], lo);
              atomicMax(&mx[acc], hi);
            }
            acc = iu[u];
            lo = INT32_MAX;
            hi = INT32_MIN;
          }
          lo = vv[u] < lo ? vv[u] : lo;
          hi = vv[u] > hi ? vv[u] : hi;
        }
      }
  }
  if (mn) flush_minmax(acc, lo, hi, mn, mx);
}

// minima (rows 0, 2, 4 of n) start at INT32_MAX, maxima (rows 1, 3, 5) at INT32_MIN
__global__ void k_fill_minmax(int32_t* mm, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 6 * n) mm[i] = ((i / n) & 1) ? INT32_MIN : INT32_MAX;
}

}  // namespace

void make_keys(const int32_t* v, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff, const int32_t* mn,
               uint32_t* keys, uint32_t* payload, const int32_t* pay_src, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_make_keys, dim3(chunk_grid(n)), dim3(NT), 0, s, v, n, ebase, n_inst, koff, mn, keys, payload,
                     pay_src);
  JP_LAUNCH_CHECK();
}

void run_ids(const uint32_t* keys, int64_t n, const int64_t* koff, const int32_t* mn, int n_inst, int32_t* E,
             int32_t* first, int32_t* vals, hipStream_t s, Arena& a, int32_t* total, const RunCarry* carry,
             int32_t* table) {
  if (n <= 0) {
    if (E) fill_i32(E, 1, 0, s);
    fill_i32(first, 1, 0, s);
    if (total) fill_i32(total, 1, 0, s);
    return;
  }
  const int64_t nb = (n + RUN_TILE - 1) / RUN_TILE;
  int32_t* offs = nullptr;
  int32_t* sums = nullptr;
  if (nb > 1) {
    sums = a.alloc<int32_t>(nb, s);
    offs = a.alloc<int32_t>(nb + 1, s);
    hipLaunchKernelGGL(k_run_heads, dim3(int(nb)), dim3(RUN_NT), 0, s, keys, n, sums);
    JP_LAUNCH_CHECK();
    scan_excl_i32(sums, offs, nb, s, a);
  }
  const RunCarry c = carry ? *carry : RunCarry{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (carry)
    hipLaunchKernelGGL(k_run_ids<RUN_CARRY>, dim3(int(nb)), dim3(RUN_NT), 0, s, keys, n, (const int32_t*)offs, koff,
                       mn, n_inst, E, first, vals, total, c, table);
  else if (E)
    hipLaunchKernelGGL(k_run_ids<RUN_E>, dim3(int(nb)), dim3(RUN_NT), 0, s, keys, n, (const int32_t*)offs, koff, mn,
                       n_inst, E, first, vals, total, c, table);
  else
    hipLaunchKernelGGL(k_run_ids<RUN_NONE>, dim3(int(nb)), dim3(RUN_NT), 0, s, keys, n, (const int32_t*)offs, koff,
                       mn, n_inst, E, first, vals, total, c, table);
  JP_LAUNCH_CHECK();
  if (nb > 1) {
    a.give_back(offs, s);
    a.give_back(sums, s);
  }
}

void ids_at_bases(const int32_t* first, const int32_t* total, const int32_t* ebase, int n_inst, int32_t* out,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_ids_at_bases, dim3((n_inst + 1 + NT - 1) / NT), dim3(NT), 0, s, first, total, ebase, n_inst,
                     out);
  JP_LAUNCH_CHECK();
}

void gather_bases(const int32_t* E, const int32_t* ebase, int n_inst, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_bases, dim3((n_inst + 1 + NT - 1) / NT), dim3(NT), 0, s, E, ebase, n_inst, out);
  JP_LAUNCH_CHECK();
}

void semijoin(const int32_t* ry, int64_t n, const int32_t* ebase, int n_inst, const int32_t* vals_y,
              const int32_t* y_base, int32_t* keep, int32_t* yid, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_semijoin, dim3(chunk_grid(n)), dim3(NT), 0, s, ry, n, ebase, n_inst, vals_y, y_base, keep, yid);
  JP_LAUNCH_CHECK();
}

void semijoin_direct(const int32_t* ry, int64_t n, const int32_t* ebase, int n_inst, const uint32_t* ykeys, int64_t ns,
                     const int32_t* first, const int32_t* total, const int64_t* koff, int64_t key_space,
                     const int32_t* mn, int32_t* table, int32_t* keep, int32_t* yid, hipStream_t s) {
  fill_i32(table, key_space, -1, s);
  if (ns > 0) {
    hipLaunchKernelGGL(k_fill_direct, dim3(grid(ns, 8192)), dim3(NT), 0, s, ykeys, first, total, table);
    JP_LAUNCH_CHECK();
  }
  if (n <= 0) return;
  hipLaunchKernelGGL(k_semijoin_direct, dim3(chunk_grid(n)), dim3(NT), 0, s, ry, n, ebase, n_inst, koff, mn, table, keep,
                     yid);
  JP_LAUNCH_CHECK();
}

void semijoin_compact(const SemiJoinIn& in, uint32_t* xk, uint32_t* oy, int32_t* rpbase, int32_t* total,
                      hipStream_t s, Arena& a) {
  if (in.n <= 0) {
    fill_i32(rpbase, int64_t(in.n_inst) + 1, 0, s);
    fill_i32(total, 1, 0, s);
    return;
  }
  const int64_t nt = (in.n + SJ_TILE - 1) / SJ_TILE;
  uint64_t* status = a.alloc<uint64_t>(nt + 2, s);
  fill_i64(reinterpret_cast<int64_t*>(status), nt + 2, 0, s);
  if (in.table)
    hipLaunchKernelGGL(k_semijoin_compact<true>, dim3(int(nt)), dim3(SJ_NT), 0, s, in, xk, oy, rpbase, total, status,
                       nt);
  else
    hipLaunchKernelGGL(k_semijoin_compact<false>, dim3(int(nt)), dim3(SJ_NT), 0, s, in, xk, oy, rpbase, total,
                       status, nt);
  JP_LAUNCH_CHECK();
  a.give_back(status, s);
}

void run_lengths(const int32_t* first, int64_t n_id, int32_t* m, hipStream_t s) {
  if (n_id <= 0) return;
  hipLaunchKernelGGL(k_run_lengths, dim3(grid(n_id)), dim3(NT), 0, s, first, n_id, m);
  JP_LAUNCH_CHECK();
}

void histogram(const uint32_t* v, int64_t n, int32_t* h, hipStream_t s, int64_t nbins) {
  if (n <= 0) return;
  if (nbins > 0 && nbins <= SMALL_BINS) {
    // about four blocks per CU, each over a long run so its flush of nbins is amortised
    const int64_t per_block = std::max<int64_t>(int64_t(16) * nbins, (n + 1023) / 1024);
    const int blocks = int((n + per_block - 1) / per_block);
    hipLaunchKernelGGL(k_histogram_small, dim3(blocks), dim3(NT), 0, s, v, n, int(nbins), per_block, h);
    JP_LAUNCH_CHECK();
    return;
  }
  const int blocks = int((n + HG_PER_BLOCK - 1) / HG_PER_BLOCK);
  hipLaunchKernelGGL(k_histogram, dim3(blocks), dim3(NT), 0, s, v, n, h);
  JP_LAUNCH_CHECK();
}

void out_j_per_inst(const int32_t* dR, const int32_t* dS, int64_t n_y, const int32_t* y_base, int n_inst,
                    int64_t* out_j, hipStream_t s) {
  fill_i64(out_j, n_inst, 0, s);
  if (n_y <= 0) return;
  hipLaunchKernelGGL(k_out_j, dim3(n_inst == 1 ? grid(n_y, 1024) : chunk_grid(n_y)), dim3(NT), 0, s, dR, dS, n_y,
                     y_base, n_inst, out_j);
  JP_LAUNCH_CHECK();
}

void key_hist(const int32_t* v, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff, const int32_t* mn,
              const int32_t* filter, int32_t* h, hipStream_t s) {
  if (n <= 0) return;
  const int blocks = int((n + HG_PER_BLOCK - 1) / HG_PER_BLOCK);
  hipLaunchKernelGGL(k_key_hist, dim3(blocks), dim3(NT), 0, s, v, n, ebase, n_inst, koff, mn, filter, h);
  JP_LAUNCH_CHECK();
}

void presence(const int32_t* cnt, int64_t n_keys, int32_t* pres, hipStream_t s) {
  if (n_keys <= 0) return;
  hipLaunchKernelGGL(k_presence, dim3(grid(n_keys)), dim3(NT), 0, s, cnt, n_keys, pres);
  JP_LAUNCH_CHECK();
}

void key_ids(const int32_t* cnt, int64_t n_keys, const int32_t* E, const int32_t* C, const int64_t* koff,
             const int32_t* mn, int n_inst, int32_t* vals, int32_t* m, int32_t* first, hipStream_t s) {
  if (n_keys <= 0) {
    if (first) fill_i32(first, 1, 0, s);
    return;
  }
  hipLaunchKernelGGL(k_key_ids, dim3(grid(n_keys)), dim3(NT), 0, s, cnt, n_keys, E, C, koff, mn, n_inst, vals, m,
                     first);
  JP_LAUNCH_CHECK();
}

void bases_from_koff(const int32_t* E, const int64_t* koff, int n_inst, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bases_from_koff, dim3((n_inst + 1 + NT - 1) / NT), dim3(NT), 0, s, E, koff, n_inst, out);
  JP_LAUNCH_CHECK();
}

void scatter_z(const int32_t* sz, const int32_t* sy, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff_z,
               const int32_t* zmin, const int64_t* koff_y, const int32_t* ymin, const int32_t* Ez, int32_t* cur,
               uint32_t* yk, uint32_t* zid, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter_z, dim3(chunk_grid(n)), dim3(NT), 0, s, sz, sy, n, ebase, n_inst, koff_z, zmin, koff_y,
                     ymin, Ez, cur, yk, zid);
  JP_LAUNCH_CHECK();
}

void scatter_x(const int32_t* rx, const int32_t* yid, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff_x,
               const int32_t* xmin, int32_t* cur, int32_t* rcol, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_scatter_x, dim3(chunk_grid(n)), dim3(NT), 0, s, rx, yid, n, ebase, n_inst, koff_x, xmin, cur,
                     rcol);
  JP_LAUNCH_CHECK();
}

void fill_minmax(int32_t* mm, int n_inst, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_minmax, dim3((6 * n_inst + 255) / 256), dim3(256), 0, s, mm, n_inst);
  JP_LAUNCH_CHECK();
}

void gather_cols(const int32_t* const* src, const int32_t* base, int n_inst, int64_t n, int32_t* dst, int32_t* mn,
                 int32_t* mx, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_cols, dim3(chunk_grid(n)), dim3(256), 0, s, src, base, n_inst, n, dst, mn, mx);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
