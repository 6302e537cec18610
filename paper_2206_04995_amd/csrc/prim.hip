// Device primitives for gfx950: single-pass scan with decoupled look-back, LSD radix sort with
// wave-ballot ranking and LDS-staged scatter, segmented min/max, fills.
#include <climits>

#include "../../include/jp.h"
#include "common.h"
#include "prim.h"

namespace jp {

namespace {

constexpr int SCAN_NT = 256;
constexpr int SCAN_IT = 8;
constexpr int SCAN_TILE = SCAN_NT * SCAN_IT;

template <class T>
__device__ T block_excl_scan(T v, T* lds, T& total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  T inc = wave_incl_scan(v);
  if (lane == 63) lds[wid] = inc;
  __syncthreads();
  T pre = 0, tot = 0;
  for (int w = 0; w < nw; ++w) {
    T s = lds[w];
    if (w < wid) pre += s;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return pre + inc - v;
}

// exclusive scan of `in` with an added per-block offset; out[n] written by the last block
template <class Ti, class To>
__global__ void __launch_bounds__(SCAN_NT) k_scan_apply(const Ti* __restrict__ in, To* __restrict__ out,
                                                        int64_t n, const To* __restrict__ offs,
                                                        int single) {
  __shared__ To lds[SCAN_NT / 64];
  int64_t base = int64_t(blockIdx.x) * SCAN_TILE + int64_t(threadIdx.x) * SCAN_IT;
  To v[SCAN_IT];
  To loc = 0;
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? To(in[i]) : To(0);
    loc += v[j];
  }
  To tot;
  To pre = block_excl_scan<To>(loc, lds, tot);
  To off = single ? To(0) : offs[blockIdx.x];
  To run = off + pre;
#pragma unroll
  for (int j = 0; j < SCAN_IT; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = off + tot;
}

// Single-pass exclusive scan with decoupled look-back (lookback_exclusive in
// common.h): the input is read once.
constexpr int LB_NT = 256;
constexpr int LB_IT = 16;
constexpr int LB_WTILE = 64 * LB_IT;    // consecutive elements per wave
constexpr int LB_TILE = LB_NT * LB_IT;  // 4096 elements per tile

template <class T>
__device__ __forceinline__ T lb_wave_incl(T v) {
  if constexpr (sizeof(T) == 4) return T(wave_scan_add_dpp(int(v)));
  else return wave_incl_scan(v);
}

template <class Ti, class To>
__global__ void __launch_bounds__(LB_NT) k_scan_lookback(const Ti* __restrict__ in, To* __restrict__ out, int64_t n,
                                                         uint64_t* __restrict__ status, int64_t ntiles) {
  __shared__ int64_t s_tile;
  __shared__ To s_wsum[LB_NT / 64];
  __shared__ To s_excl;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_tile = lookback_ticket(status, ntiles);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t w0 = tile * LB_TILE + int64_t(wid) * LB_WTILE;
  To v[LB_IT];
#pragma unroll
  for (int j = 0; j < LB_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    v[j] = i < n ? To(in[i]) : To(0);
  }
  To run = 0;  // wave-uniform
#pragma unroll
  for (int j = 0; j < LB_IT; ++j) {
    const To inc = lb_wave_incl<To>(v[j]);
    const To ex = run + inc - v[j];
    run += __shfl(inc, 63, 64);
    v[j] = ex;
  }
  if (lane == 0) s_wsum[wid] = run;
  __syncthreads();
  To woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < LB_NT / 64; ++w) {
    if (w < wid) woff += s_wsum[w];
    btot += s_wsum[w];
  }
  if (wid == 0) {
    const To excl = To(lookback_exclusive(status, tile, ntiles, int64_t(btot)));
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  const To base = s_excl + woff;
#pragma unroll
  for (int j = 0; j < LB_IT; ++j) {
    const int64_t i = w0 + j * 64 + lane;
    if (i < n) out[i] = base + v[j];
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) out[n] = s_excl + btot;
}

template <class Ti, class To>
void scan_impl(const Ti* in, To* out, int64_t n, hipStream_t s, Arena& a) {
  if (n <= 0) {
    hipLaunchKernelGGL((k_scan_apply<Ti, To>), dim3(1), dim3(SCAN_NT), 0, s, in, out, int64_t(0),
                       (const To*)nullptr, 1);
    JP_LAUNCH_CHECK();
    return;
  }
  if (n <= SCAN_TILE) {
    hipLaunchKernelGGL((k_scan_apply<Ti, To>), dim3(1), dim3(SCAN_NT), 0, s, in, out, n,
                       (const To*)nullptr, 1);
    JP_LAUNCH_CHECK();
    return;
  }
  const int64_t nt = (n + LB_TILE - 1) / LB_TILE;
  uint64_t* status = a.alloc<uint64_t>(nt + 2, s);  // tile words, the tile counter, a give-up flag
  fill_i64(reinterpret_cast<int64_t*>(status), nt + 2, 0, s);
  hipLaunchKernelGGL((k_scan_lookback<Ti, To>), dim3(int(nt)), dim3(LB_NT), 0, s, in, out, n, status, nt);
  JP_LAUNCH_CHECK();
  a.give_back(status, s);
}

// ------------------------------------------------------------ radix sort

constexpr int RS_NT = 256;
constexpr int RS_IT = 16;
constexpr int RS_TILE = RS_NT * RS_IT;  // 4096 keys per block
constexpr int RS_WAVES = RS_NT / 64;
constexpr int RS_WTILE = RS_TILE / RS_WAVES;  // 1024 keys per wave
// Digits are at most 8 bits wide.  (9-bit digits, two passes instead of
// three for a 17-bit range, were slower: with 4096-key tiles a 512-way
// scatter writes runs of about 8 keys.)
constexpr int RS_MAXBITS = 8;
constexpr int RS_MAXD = 1 << RS_MAXBITS;
constexpr int RS_SUB = 4;  // digit counter sets per wave in the histogram pass

// Tiles of a segmented sort: segment i (elements [ebase[i], ebase[i+1]), keys
// in [koff[i], koff[i] + 2^bits)) owns tiles [toff[i], toff[i+1]), so no tile
// spans two segments.  The histogram of tile t of segment i, digit d, sits at
// toff[i] * nd + d * T_i + (t - toff[i]) (T_i tiles): a flat scan then orders
// the output by segment, digit, tile, which keeps every segment in place.  A
// plain sort is one segment with koff 0.
struct TileMap {
  const int32_t* toff;   // [n_seg + 1]
  const int32_t* ebase;  // [n_seg + 1]
  const int64_t* koff;   // [n_seg] (null: 0)
  int n_seg;             // 0: one segment [0, n)
  const int32_t* mn;     // raw input (first pass only): key = koff + value - mn of the segment
  // raw input in one buffer per segment (first pass only, n_seg > 0): element
  // i of segment s is rk[s][i - ebase[s]] (values rv[s][...]); null: the
  // pass's input arrays
  const int32_t* const* rk;
  const int32_t* const* rv;
};

struct Tile {
  int64_t lo, hi;   // elements
  int64_t hbase;    // histogram index of digit 0
  int stride;       // histogram distance of consecutive digits (tiles of the segment)
  int64_t koff;     // subtracted from the keys
  int64_t radd;     // raw input: added to a value to give its key
  const uint32_t* kp;  // raw input in the segment's own buffer (null: the pass's input array)
  const uint32_t* vp;
  int64_t e0;          // the segment's first element (index 0 of kp, vp)
};

// whole wave, uniform control flow
__device__ __forceinline__ Tile tile_of(const TileMap& m, int64_t n, int nd) {
  Tile t;
  const int b = blockIdx.x;
  if (m.n_seg == 0) {
    t.lo = int64_t(b) * RS_TILE;
    t.hi = t.lo + RS_TILE < n ? t.lo + RS_TILE : n;
    t.hbase = b;
    t.stride = int(gridDim.x);
    t.koff = 0;
    t.radd = m.mn ? (m.koff ? m.koff[0] : 0) - int64_t(m.mn[0]) : 0;
    t.kp = nullptr;
    t.vp = nullptr;
    t.e0 = 0;
    return t;
  }
  const int sg = wave_find_inst<int32_t>(m.toff, m.n_seg, b);
  const int t0 = m.toff[sg], nt = m.toff[sg + 1] - t0;
  const int64_t e1 = m.ebase[sg + 1];
  t.lo = int64_t(m.ebase[sg]) + int64_t(b - t0) * RS_TILE;
  t.hi = t.lo + RS_TILE < e1 ? t.lo + RS_TILE : e1;
  t.hbase = int64_t(t0) * nd + (b - t0);
  t.stride = nt;
  t.koff = m.koff ? m.koff[sg] : 0;
  t.radd = m.mn ? t.koff - int64_t(m.mn[sg]) : 0;
  t.kp = m.rk ? reinterpret_cast<const uint32_t*>(m.rk[sg]) : nullptr;
  t.vp = m.rv ? reinterpret_cast<const uint32_t*>(m.rv[sg]) : nullptr;
  t.e0 = m.ebase[sg];
  return t;
}

// a loaded element's key: raw values are moved into the segment's key range
template <bool RAW>
__device__ __forceinline__ uint32_t key_in(uint32_t k, const Tile& t) {
  return RAW ? uint32_t(int64_t(int32_t(k)) + t.radd) : k;
}

__device__ __forceinline__ uint32_t digit_of(uint32_t k, const Tile& t, int shift, uint32_t mask) {
  return (uint32_t(int64_t(k) - t.koff) >> shift) & mask;
}

// Lanes of one wave row whose keys share digit d: the ballots of d's bits
// (a lane's own mask, lowest lane = the group's leader).
__device__ __forceinline__ uint64_t digit_match(uint32_t d, bool valid, int nbits) {
  uint64_t m = ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bb = ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

template <bool RAW>
__global__ void __launch_bounds__(RS_NT) k_radix_hist(const uint32_t* __restrict__ keys, int64_t n,
                                                       int shift, int nbits, int* __restrict__ hist,
                                                       TileMap m) {
  __shared__ int cnt[RS_WAVES * RS_SUB][RS_MAXD];
  const int wid = threadIdx.x >> 6;
  const int nd = 1 << nbits;
  const uint32_t mask = uint32_t(nd - 1);
  const Tile tl = tile_of(m, n, nd);
  for (int i = threadIdx.x; i < RS_WAVES * RS_SUB * RS_MAXD; i += RS_NT) (&cnt[0][0])[i] = 0;
  __syncthreads();
  // all of a thread's loads first (clamped, so they need no branch), then the LDS counts
  const bool own = RAW && tl.kp;  // raw input in the segment's own buffer
  const uint32_t* kb = own ? tl.kp : keys;
  const int64_t ko = own ? tl.e0 : 0;
  uint32_t kk[RS_IT];
#pragma unroll
  for (int j = 0; j < RS_IT; ++j) {
    const int64_t i = tl.lo + j * RS_NT + threadIdx.x;
    kk[j] = key_in<RAW>(kb[(i < tl.hi ? i : tl.hi - 1) - ko], tl);
  }
  // four counter sets per wave (by lane mod 4): concentrated digits (the high
  // digits of clustered keys) put at most 16 lanes of a row on one counter
  const int sub = wid * RS_SUB + (lane_id() & (RS_SUB - 1));
#pragma unroll
  for (int j = 0; j < RS_IT; ++j)
    if (tl.lo + j * RS_NT + threadIdx.x < tl.hi) atomicAdd(&cnt[sub][digit_of(kk[j], tl, shift, mask)], 1);
  __syncthreads();
  for (int d = threadIdx.x; d < nd; d += RS_NT) {
    int c = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES * RS_SUB; ++w) c += cnt[w][d];
    hist[tl.hbase + int64_t(d) * tl.stride] = c;
  }
}

// T_i = tiles of segment i
__global__ void k_tile_counts(const int32_t* __restrict__ ebase, int n_seg, int32_t* __restrict__ cnt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n_seg) cnt[i] = int32_t((int64_t(ebase[i + 1]) - ebase[i] + RS_TILE - 1) / RS_TILE);
}

template <bool HAS_V, bool RAW>
__global__ void __launch_bounds__(RS_NT) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout, int64_t n,
                                                          int shift, int nbits,
                                                          const int* __restrict__ offs, TileMap m) {
  __shared__ uint32_t s_k[RS_TILE];
  __shared__ uint32_t s_v[HAS_V ? RS_TILE : 1];
  __shared__ int wcnt[RS_WAVES][RS_MAXD];
  __shared__ int dstart[RS_MAXD];
  __shared__ int goff[RS_MAXD];
  __shared__ int scan_lds[RS_NT / 64];
  static_assert(RS_MAXD <= RS_NT, "one thread per digit in the digit scan");

  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int nd = 1 << nbits;
  const uint32_t mask = uint32_t(nd - 1);
  const uint64_t ltm = lanemask_lt();
  const Tile tl = tile_of(m, n, nd);
  for (int i = threadIdx.x; i < RS_WAVES * RS_MAXD; i += RS_NT) (&wcnt[0][0])[i] = 0;
  __syncthreads();

  const int64_t wbase = tl.lo + int64_t(wid) * RS_WTILE;
  const bool own = RAW && tl.kp;  // raw input in the segment's own buffers
  const uint32_t* kb = own ? tl.kp : kin;
  const uint32_t* vb = own ? tl.vp : vin;
  const int64_t ko = own ? tl.e0 : 0;
  uint32_t key[RS_IT], val[RS_IT];
#pragma unroll
  for (int j = 0; j < RS_IT; ++j) {
    const int64_t i = wbase + j * 64 + lane;
    const bool valid = i < tl.hi;
    key[j] = valid ? kb[i - ko] : 0u;
    if (HAS_V) val[j] = valid ? vb[i - ko] : 0u;
  }
  // raw values become keys only once every load is in flight (converting each
  // as it arrives would make the loads wait for one another); lanes past the
  // tile end are never ranked, whatever their key
  if (RAW) {
#pragma unroll
    for (int j = 0; j < RS_IT; ++j) key[j] = key_in<RAW>(key[j], tl);
  }
  // Stable ranks inside the wave: per row, the group leader of each digit adds
  // the group's size to the wave's counter and gets the count before it.  The
  // adds of all rows are issued back to back; LDS executes one wave's
  // operations in order, so row j sees the counts of rows before it.
  int before[RS_IT], lead[RS_IT], lrank[RS_IT];
#pragma unroll
  for (int j = 0; j < RS_IT; ++j) {
    const bool valid = wbase + j * 64 + lane < tl.hi;
    const uint32_t d = digit_of(key[j], tl, shift, mask);
    const uint64_t mm = digit_match(d, valid, nbits);
    lead[j] = valid ? __ffsll((unsigned long long)mm) - 1 : lane;
    lrank[j] = valid ? __popcll(mm & ltm) : -1;
    before[j] = 0;
    if (valid && lane == lead[j]) before[j] = atomicAdd(&wcnt[wid][d], __popcll(mm));
  }
#pragma unroll
  for (int j = 0; j < RS_IT; ++j) {
    const int b = __shfl(before[j], lead[j], 64);  // every lane takes part
    if (lrank[j] >= 0) lrank[j] += b;
  }
  __syncthreads();
  // per digit: prefix across waves, block total, block-local start
  int tot_d = 0;
  if (threadIdx.x < nd) {
    int run = 0;
#pragma unroll
    for (int w = 0; w < RS_WAVES; ++w) {
      int c = wcnt[w][threadIdx.x];
      wcnt[w][threadIdx.x] = run;
      run += c;
    }
    tot_d = run;
    goff[threadIdx.x] = offs[tl.hbase + int64_t(threadIdx.x) * tl.stride];
  }
  int tile_total;
  int st = block_excl_scan<int>(tot_d, scan_lds, tile_total);
  if (threadIdx.x < nd) dstart[threadIdx.x] = st;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < RS_IT; ++j) {
    if (lrank[j] >= 0) {
      uint32_t d = digit_of(key[j], tl, shift, mask);
      int pos = dstart[d] + wcnt[wid][d] + lrank[j];
      s_k[pos] = key[j];
      if (HAS_V) s_v[pos] = val[j];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < tile_total; i += RS_NT) {
    uint32_t k = s_k[i];
    uint32_t d = digit_of(k, tl, shift, mask);
    int64_t g = int64_t(goff[d]) + (i - dstart[d]);
    kout[g] = k;
    if (HAS_V) vout[g] = s_v[i];
  }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Per-segment min and max.  A block owns a contiguous chunk of MM_CHUNK
// elements read with coalesced, strided loads.  When the chunk lies in one
// segment (the common case: few, large segments) the block reduces through
// LDS and issues one atomic pair; otherwise each thread tracks the segment of
// its (increasing) elements and flushes at every change.
constexpr int MM_NT = 256;
constexpr int MM_CHUNK = MM_NT * 64;

__global__ void __launch_bounds__(MM_NT) k_seg_minmax(const int32_t* __restrict__ v, int64_t n,
                                                      const int32_t* __restrict__ base, int n_seg,
                                                      int32_t* __restrict__ mn, int32_t* __restrict__ mx) {
  __shared__ int32_t s_mn[MM_NT / 64], s_mx[MM_NT / 64];
  const int64_t c0 = int64_t(blockIdx.x) * MM_CHUNK;
  const int64_t c1 = c0 + MM_CHUNK < n ? c0 + MM_CHUNK : n;
  const int seg0 = wave_find_inst<int32_t>(base, n_seg, int32_t(c0));
  const int seg1 = wave_find_inst<int32_t>(base, n_seg, int32_t(c1 - 1));
  int32_t cmn = INT_MAX, cmx = INT_MIN;
  if (seg0 == seg1) {
#pragma unroll 8  // independent loads in flight: one at a time leaves each thread waiting on memory
    for (int64_t i = c0 + threadIdx.x; i < c1; i += MM_NT) {
      const int32_t x = v[i];
      cmn = x < cmn ? x : cmn;
      cmx = x > cmx ? x : cmx;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const int32_t a = __shfl_xor(cmn, o, 64), b = __shfl_xor(cmx, o, 64);
      cmn = a < cmn ? a : cmn;
      cmx = b > cmx ? b : cmx;
    }
    if (lane_id() == 0) {
      s_mn[threadIdx.x >> 6] = cmn;
      s_mx[threadIdx.x >> 6] = cmx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < MM_NT / 64; ++w) {
        cmn = s_mn[w] < cmn ? s_mn[w] : cmn;
        cmx = s_mx[w] > cmx ? s_mx[w] : cmx;
      }
      atomicMin(&mn[seg0], cmn);
      atomicMax(&mx[seg0], cmx);
    }
    return;
  }
  int seg = seg0;
  bool any = false;
  for (int64_t i = c0 + threadIdx.x; i < c1; i += MM_NT) {
    while (i >= base[seg + 1]) {
      if (any) {
        atomicMin(&mn[seg], cmn);
        atomicMax(&mx[seg], cmx);
      }
      any = false;
      cmn = INT_MAX;
      cmx = INT_MIN;
      ++seg;
    }
    const int32_t x = v[i];
    cmn = x < cmn ? x : cmn;
    cmx = x > cmx ? x : cmx;
    any = true;
  }
  if (any) {
    atomicMin(&mn[seg], cmn);
    atomicMax(&mx[seg], cmx);
  }
}

__global__ void k_reduce_sum_i32(const int32_t* __restrict__ a, int64_t n, int64_t* out) {
  int64_t acc = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    acc += a[i];
  acc = wave_sum(acc);
  if (lane_id() == 0 && acc) atomicAdd((unsigned long long*)out, (unsigned long long)acc);
}

int grid_for(int64_t n, int nt = 256, int cap = 65536) {
  int64_t g = (n + nt - 1) / nt;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

}  // namespace

int bits_for(uint64_t range) {
  int b = 0;
  while (b < 64 && (uint64_t(1) << b) < range) ++b;
  return b;
}

void scan_excl_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s, Arena& a) {
  scan_impl<int32_t, int32_t>(in, out, n, s, a);
}
void scan_excl_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s, Arena& a) {
  scan_impl<int32_t, int64_t>(in, out, n, s, a);
}
void scan_excl_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s, Arena& a) {
  scan_impl<int64_t, int64_t>(in, out, n, s, a);
}

int radix_passes(int64_t n, int bits) {
  return (n <= 1 || bits <= 0) ? 0 : (bits + RS_MAXBITS - 1) / RS_MAXBITS;
}

namespace {

void launch_hist(bool raw, int nblocks, const uint32_t* ki, int64_t n, int shift, int w, int* hist,
                 const TileMap& m, hipStream_t s) {
  if (raw)
    hipLaunchKernelGGL((k_radix_hist<true>), dim3(nblocks), dim3(RS_NT), 0, s, ki, n, shift, w, hist, m);
  else
    hipLaunchKernelGGL((k_radix_hist<false>), dim3(nblocks), dim3(RS_NT), 0, s, ki, n, shift, w, hist, m);
  JP_LAUNCH_CHECK();
}

void launch_scatter(bool raw, bool has_v, int nblocks, const uint32_t* ki, const uint32_t* vi, uint32_t* ko,
                    uint32_t* vo, int64_t n, int shift, int w, const int* offs, const TileMap& m, hipStream_t s) {
  if (!has_v) {
    vi = nullptr;
    vo = nullptr;
  }
  if (raw && has_v)
    hipLaunchKernelGGL((k_radix_scatter<true, true>), dim3(nblocks), dim3(RS_NT), 0, s, ki, vi, ko, vo, n,
                       shift, w, offs, m);
  else if (raw)
    hipLaunchKernelGGL((k_radix_scatter<false, true>), dim3(nblocks), dim3(RS_NT), 0, s, ki, vi, ko, vo, n,
                       shift, w, offs, m);
  else if (has_v)
    hipLaunchKernelGGL((k_radix_scatter<true, false>), dim3(nblocks), dim3(RS_NT), 0, s, ki, vi, ko, vo, n,
                       shift, w, offs, m);
  else
    hipLaunchKernelGGL((k_radix_scatter<false, false>), dim3(nblocks), dim3(RS_NT), 0, s, ki, vi, ko, vo, n,
                       shift, w, offs, m);
  JP_LAUNCH_CHECK();
}

// The passes of a sort whose first pass reads (k0, v0): (k, v) itself, or raw
// values moved into their segments' key ranges by raw_mn.
bool radix_impl(const uint32_t* k0, const uint32_t* v0, const int32_t* raw_mn, const int32_t* const* seg_k,
                const int32_t* const* seg_v, uint32_t* k, uint32_t* v, uint32_t* kt, uint32_t* vt, int64_t n,
                int bits, hipStream_t s, Arena& a, const SortSegments* seg) {
  if (n <= 1 || bits <= 0) return false;
  int passes = radix_passes(n, bits);
  int width = (bits + passes - 1) / passes;
  TileMap m{nullptr, nullptr, raw_mn && seg ? seg->d_koff : nullptr, 0, raw_mn, nullptr, nullptr};
  int nblocks = int((n + RS_TILE - 1) / RS_TILE);
  int32_t* toff = nullptr;
  if (seg && seg->n_seg > 1) {
    const int ns = seg->n_seg;
    int64_t nb = 0;
    for (int i = 0; i < ns; ++i) nb += (seg->h_ebase[i + 1] - seg->h_ebase[i] + RS_TILE - 1) / RS_TILE;
    nblocks = int(nb);
    int32_t* tc = a.alloc<int32_t>(ns, s);
    toff = a.alloc<int32_t>(ns + 1, s);
    hipLaunchKernelGGL(k_tile_counts, dim3((ns + 255) / 256), dim3(256), 0, s, seg->d_ebase, ns, tc);
    JP_LAUNCH_CHECK();
    scan_excl_i32(tc, toff, ns, s, a);
    a.give_back(tc, s);
    m = TileMap{toff, seg->d_ebase, seg->d_koff, ns, raw_mn, seg_k, seg_v};
  } else if (seg_k) {
    throw Error(JP_EINVAL, "per-segment input needs more than one segment");
  }
  if (nblocks == 0) return false;
  int64_t hsz = int64_t(1 << width) * nblocks;
  int* hist = a.alloc<int>(hsz, s);
  int* offs = a.alloc<int>(hsz + 1, s);
  const uint32_t *ki = k0, *vi = v0;
  uint32_t *ko = kt, *vo = vt;
  int shift = 0;
  for (int p = 0; p < passes; ++p) {
    int w = width;
    if (shift + w > bits) w = bits - shift;
    const bool raw = m.mn != nullptr;
    launch_hist(raw, nblocks, ki, n, shift, w, hist, m, s);
    scan_impl<int, int>(hist, offs, int64_t(1 << w) * nblocks, s, a);
    launch_scatter(raw, v != nullptr, nblocks, ki, vi, ko, vo, n, shift, w, offs, m, s);
    m.mn = nullptr;
    m.rk = nullptr;
    m.rv = nullptr;
    // the pass wrote (ko, vo); the next one writes the other pair
    uint32_t* nk = ko == kt ? k : kt;
    uint32_t* nv = ko == kt ? v : vt;
    ki = ko;
    vi = vo;
    ko = nk;
    vo = nv;
    shift += w;
  }
  a.give_back(offs, s);
  a.give_back(hist, s);
  if (toff) a.give_back(toff, s);
  return ki == kt;
}

}  // namespace

bool radix_sort_pairs(uint32_t* k, uint32_t* v, uint32_t* kt, uint32_t* vt, int64_t n, int bits,
                      hipStream_t s, Arena& a, const SortSegments* seg) {
  return radix_impl(k, v, nullptr, nullptr, nullptr, k, v, kt, vt, n, bits, s, a, seg);
}

bool radix_sort_raw(const int32_t* raw, const int32_t* raw_v, const int32_t* const* seg_raw,
                    const int32_t* const* seg_raw_v, const int32_t* mn, uint32_t* k, uint32_t* v, uint32_t* kt,
                    uint32_t* vt, int64_t n, int bits, hipStream_t s, Arena& a, const SortSegments& seg) {
  if (radix_passes(n, bits) == 0) throw Error(JP_EINVAL, "radix_sort_raw needs at least one pass");
  if (seg_raw && v && !seg_raw_v) throw Error(JP_EINVAL, "radix_sort_raw: keys per segment need values per segment");
  return radix_impl(reinterpret_cast<const uint32_t*>(raw), reinterpret_cast<const uint32_t*>(raw_v), mn, seg_raw,
                    seg_raw_v, k, v, kt, vt, n, bits, s, a, &seg);
}

void seg_minmax(const int32_t* v, int64_t n, const int32_t* base, int n_seg, int32_t* mn, int32_t* mx,
                hipStream_t s) {
  fill_i32(mn, n_seg, INT_MAX, s);
  fill_i32(mx, n_seg, INT_MIN, s);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_seg_minmax, dim3(int((n + MM_CHUNK - 1) / MM_CHUNK)), dim3(MM_NT), 0, s, v, n, base, n_seg,
                     mn, mx);
  JP_LAUNCH_CHECK();
}

void fill_i32(int32_t* p, int64_t n, int32_t val, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, p, n, val);
  JP_LAUNCH_CHECK();
}
void fill_i64(int64_t* p, int64_t n, int64_t val, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n)), dim3(256), 0, s, p, n, val);
  JP_LAUNCH_CHECK();
}
void fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, s, p, n, val);
  JP_LAUNCH_CHECK();
}

void reduce_sum_i32_to_i64(const int32_t* a, int64_t n, int64_t* out, hipStream_t s) {
  fill_i64(out, 1, 0, s);
  if (n <= 0) return;
  hipLaunchKernelGGL(k_reduce_sum_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, a, n, out);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
