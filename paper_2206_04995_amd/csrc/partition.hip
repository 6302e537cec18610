// Intersection-free partition of S by z (paper Sec. 2.3, Alg. 1): every S
// tuple of a z goes to the dense part iff
// m_z > tau for that z's instance, so the results of the two parts are
// disjoint.  Also builds the structures of the dense part: the hot join keys
// (y with many dense S entries) as bit rows over the dense z index, and the
// remaining dense entries as "cold" CSR rows.
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

__global__ void k_dense_flags(const int32_t* __restrict__ m_z, int64_t n_z, const int32_t* __restrict__ z_base,
                              int n_inst, const int64_t* __restrict__ tau, int32_t* __restrict__ flag) {
  SegCursor<int32_t> zcur(z_base, n_inst);
  zcur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(z, n_z, JP_CHUNK) {
    const int inst = zcur(int32_t(z));
    flag[z] = int64_t(m_z[z]) > tau[inst] ? 1 : 0;
  }
}

__global__ void k_dense_index(const int32_t* __restrict__ flag, const int32_t* __restrict__ Edz, int64_t n_z,
                              int32_t* __restrict__ dz2z) {
  GRID_STRIDE(z, n_z) {
    if (flag[z]) dz2z[Edz[z]] = int32_t(z);
  }
}

__global__ void k_remap_rowptr(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ E, int64_t n_y,
                               int32_t* __restrict__ out) {
  GRID_STRIDE(y, n_y + 1) { out[y] = E[rowptr[y]]; }
}

__device__ __forceinline__ int ilog2(int v) { return 31 - __clz(v); }

// entries of key y in the space: a[y+1] - a[y] - (b ? b[y+1] - b[y] : 0)
__device__ __forceinline__ int space_count(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t y) {
  return (a[y + 1] - a[y]) - (b ? b[y + 1] - b[y] : 0);
}

// Per-instance histogram of floor(log2(count in the space)) over y with dR > 0.
// A block takes a chunk of y ids (CHUNK_LOOP); counts of the chunk's first
// instance gather in LDS (one atomic per bucket and block at the end), the
// rare ids of later instances in the chunk go straight to global memory.
__global__ void k_hot_histogram(const int32_t* __restrict__ cnt_a, const int32_t* __restrict__ cnt_b,
                                const int32_t* __restrict__ dR, int64_t n_y, const int32_t* __restrict__ y_base,
                                int n_inst, int32_t* __restrict__ hist) {
  __shared__ int32_t loc[32];
  if (threadIdx.x < 32) loc[threadIdx.x] = 0;
  SegCursor<int32_t> ycur(y_base, n_inst);
  ycur.seed(int32_t(chunk_first() < n_y ? chunk_first() : 0));
  const int i0 = ycur.cur;
  __syncthreads();
  CHUNK_LOOP(y, n_y, JP_CHUNK) {
    const int dd = space_count(cnt_a, cnt_b, y);
    if (dd > 0 && dR[y] > 0) {
      const int inst = ycur(int32_t(y));
      if (inst == i0) atomicAdd(&loc[ilog2(dd)], 1);
      else atomicAdd(&hist[inst * 32 + ilog2(dd)], 1);
    }
  }
  __syncthreads();
  if (threadIdx.x < 32 && loc[threadIdx.x]) atomicAdd(&hist[(i0 > 0 ? i0 : 0) * 32 + threadIdx.x], loc[threadIdx.x]);
}

__global__ void k_hot_flags(const int32_t* __restrict__ cnt_a, const int32_t* __restrict__ cnt_b,
                            const int32_t* __restrict__ dR, int64_t n_y, const int32_t* __restrict__ y_base,
                            int n_inst, const int64_t* __restrict__ theta, int32_t* __restrict__ hot) {
  SegCursor<int32_t> ycur(y_base, n_inst);
  ycur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(y, n_y, JP_CHUNK) {
    const int dd = space_count(cnt_a, cnt_b, y);
    const int inst = ycur(int32_t(y));
    hot[y] = (dd > 0 && dR[y] > 0 && int64_t(dd) >= theta[inst]) ? 1 : 0;
  }
}

// Bit rows of the hot keys: one lane per entry of a hot row (the rows of the
// hot list, in list order, concatenated; hoff = their scanned lengths), which
// sets the bit of the entry's z if it lies in the space (zmap[z] = local index
// in the space, or -1).  Only hot rows are read, not every S entry.  Per hot
// key, k_hot_row_info first stores what its entries share: the distance from
// a position in the concatenation to the entry's position in S (pdel) and the
// key's first bitmap word (rbase), so an entry costs two dependent loads
// (scol, zmap).  A lane takes HU entries per step with every load issued
// before any is used.  A row's entries ascend in z, so neighbouring lanes
// often target the same word: the wave ORs the bits of lanes with equal word
// addresses (shuffle-down doubling; every bit a lane takes belongs to its own
// address) and only the first lane of each run issues the atomic.  Blocks
// stride over chunks of the concatenation (its length is known only on the
// device) and walk each chunk in wave-uniform steps, so the shuffles never
// read an inactive lane.
__global__ void k_hot_row_lengths(const int32_t* __restrict__ hotlist, int64_t n_hot,
                                  const int32_t* __restrict__ sptr, int32_t* __restrict__ len) {
  GRID_STRIDE(i, n_hot) {
    const int32_t y = hotlist[i];
    len[i] = sptr[y + 1] - sptr[y];
  }
}

__global__ void k_hot_row_info(const int32_t* __restrict__ hotlist, int64_t n_hot, const int32_t* __restrict__ hoff,
                               const int32_t* __restrict__ sptr, const int32_t* __restrict__ hotrow,
                               const int32_t* __restrict__ y_base, int n_inst, const int64_t* __restrict__ hb_off,
                               const int32_t* __restrict__ row_words, int32_t* __restrict__ pdel,
                               int64_t* __restrict__ rbase) {
  GRID_STRIDE(i, n_hot) {
    const int32_t y = hotlist[i];
    const int inst = n_inst == 1 ? 0 : find_inst<int32_t>(y_base, n_inst, y);
    pdel[i] = sptr[y] - hoff[i];
    rbase[i] = hb_off[inst] + int64_t(hotrow[y]) * row_words[inst];
  }
}

constexpr int HU = 8;  // entries per lane and step

__global__ void k_build_hot_bits(const int32_t* __restrict__ hoff, int n_hot, const int32_t* __restrict__ pdel,
                                 const int64_t* __restrict__ rbase, const int32_t* __restrict__ scol,
                                 const int32_t* __restrict__ zmap, uint32_t* __restrict__ hb) {
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const int64_t total = hoff[n_hot];
  constexpr uint64_t NONE = ~uint64_t(0);
  for (int64_t c0 = int64_t(blockIdx.x) * JP_CHUNK; c0 < total; c0 += int64_t(gridDim.x) * JP_CHUNK) {
    const int64_t c1 = c0 + JP_CHUNK < total ? c0 + JP_CHUNK : total;
    SegCursor<int32_t> hcur(hoff, n_hot);
    hcur.seed(int32_t(c0));
    for (int64_t base = c0 + int64_t(wid) * 64 * HU; base < c1; base += int64_t(blockDim.x) * HU) {
      // positions past the chunk end are clamped to its last one (valid loads) and dropped below
      int32_t ii[HU], p[HU], dl[HU];
      int64_t rb[HU];
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        const int64_t q = base + u * 64 + lane;
        const int32_t qc = int32_t(q < c1 ? q : c1 - 1);
        ii[u] = hcur(qc);
        p[u] = qc;
      }
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        p[u] += pdel[ii[u]];
        rb[u] = rbase[ii[u]];
      }
#pragma unroll
      for (int u = 0; u < HU; ++u) dl[u] = scol[p[u]];
#pragma unroll
      for (int u = 0; u < HU; ++u) dl[u] = zmap[dl[u]];
#pragma unroll
      for (int u = 0; u < HU; ++u) {
        const bool in = base + u * 64 + lane < c1 && dl[u] >= 0;
        if (ballot(in) == 0) continue;  // nothing in the space among these 64 (wave-uniform)
        uint64_t addr = in ? uint64_t(rb[u] + (dl[u] >> 5)) : NONE;
        uint32_t bits = in ? 1u << (dl[u] & 31) : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint64_t a2 = __shfl_down(addr, o, 64);
          const uint32_t b2 = __shfl_down(bits, o, 64);
          if (lane + o < 64 && a2 == addr) bits |= b2;
        }
        const uint64_t ap = __shfl_up(addr, 1, 64);
        if (addr != NONE && (lane == 0 || ap != addr)) atomicOr(&hb[addr], bits);
      }
    }
  }
}

// per S entry: 1 iff its z lies in the space
__global__ void k_space_flags(const int32_t* __restrict__ scol, int64_t n, const int32_t* __restrict__ zmap,
                              int32_t* __restrict__ flag) {
  GRID_STRIDE(p, n) flag[p] = zmap[scol[p]] >= 0 ? 1 : 0;
}

// S entries (CSR by y, the row of entry p is Ey[p + 1] - 1) filtered into a
// CSR over the same rows in one pass: the kept entries in order (out), the
// row pointers (rowptr[row] at each row's first entry, rowptr[n_rows] = kept)
// and the kept count.  A tile places its kept entries at the look-back
// prefix of the kept counts (lookback_exclusive).  Every row has an entry.
//   FILTER_SPARSE  keep z with zsel[z] == 0 (z not dense), out = z;
//   FILTER_COLD    keep z with zsel[z] >= 0 (z in the space) whose row is not
//                  hot, out = zsel[z] (the local index in the space).
constexpr int FR_NT = 512;  // 8192-entry tiles: half the look-backs of 4096
constexpr int FR_IT = 16;
constexpr int FR_WTILE = 64 * FR_IT;
constexpr int FR_TILE = FR_NT * FR_IT;
enum FilterMode { FILTER_SPARSE = 0, FILTER_COLD = 1 };

// One bit per z of the filter's z test (kept iff set).  In bits the test of a
// random z reads a table 32 times smaller than the int32 one, which mostly
// stays in cache.
//   FILTER_SPARSE  bit z of the 64-bit word zbit[z / 64];
//   FILTER_COLD    bit z % 32 of the low half of zbit[z / 32], whose high half
//                  holds the word's rank base r: every z of the word in the
//                  space has zsel[z] = r + (bits of the word below z), or r is
//                  -1 (the local indices restart inside the word, at an
//                  instance boundary) and zsel[z] is read instead.  A kept
//                  entry's local index then costs no gather from zsel.
template <int MODE>
__global__ void k_filter_bits(const int32_t* __restrict__ zsel, int64_t n_z, uint64_t* __restrict__ zbit) {
  const int lane = lane_id();
  for (int64_t base = (int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63)); base < n_z;
       base += int64_t(gridDim.x) * blockDim.x) {
    const int64_t z = base + lane;
    const int32_t v = z < n_z ? zsel[z] : -1;
    const bool k = z < n_z && (MODE == FILTER_SPARSE ? v == 0 : v >= 0);
    const uint64_t b = ballot(k);
    if (MODE == FILTER_SPARSE) {
      if (lane == 0) zbit[base >> 6] = b;
    } else {
      const int half = lane >> 5;
      const uint32_t bits = uint32_t(b >> (32 * half));
      const int32_t pred = v - __popc(bits & ((1u << (lane & 31)) - 1u));  // the base this z implies
      const int first = bits ? 32 * half + __ffs(bits) - 1 : lane;
      const int32_t p0 = __shfl(pred, first, 64);
      const uint64_t bad = ballot(k && pred != p0);
      const bool ok = uint32_t(bad >> (32 * half)) == 0u;
      const int32_t r = bits == 0u ? 0 : (ok ? p0 : -1);
      if ((lane & 31) == 0 && base + 32 * half < n_z)  // the word exists ((n_z + 31) / 32 words)
        zbit[(base >> 5) + half] = uint64_t(bits) | (uint64_t(uint32_t(r)) << 32);
    }
  }
}

template <int MODE>
__global__ void __launch_bounds__(FR_NT) k_filter_rows(const int32_t* __restrict__ Ey, const int32_t* __restrict__ scol,
                                                       int64_t n, const int32_t* __restrict__ zsel,
                                                       const uint64_t* __restrict__ zbit,
                                                       const int32_t* __restrict__ hot, int32_t* __restrict__ out,
                                                       int32_t* __restrict__ orow, int32_t* __restrict__ rowptr,
                                                       int64_t n_rows,
                                                       int32_t* __restrict__ total, uint64_t* __restrict__ status,
                                                       int64_t ntiles) {
  __shared__ int64_t s_tile;
  __shared__ int32_t s_wsum[FR_NT / 64];
  __shared__ int64_t s_excl;
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  const uint64_t ltm = lanemask_lt();
  if (threadIdx.x == 0) s_tile = lookback_ticket(status, ntiles);
  __syncthreads();
  const int64_t tile = s_tile;
  const int64_t w0 = tile * FR_TILE + int64_t(wid) * FR_WTILE;
  // every load first, at clamped (valid) indices, so the gathers of all rows are in flight together
  int32_t z[FR_IT], e1[FR_IT];
  const int32_t ew = Ey[w0 < n ? w0 : n - 1];  // the row count before the wave's first entry
#pragma unroll
  for (int j = 0; j < FR_IT; ++j) {
    int64_t i = w0 + j * 64 + lane;
    i = i < n ? i : n - 1;
    e1[j] = Ey[i + 1];
    z[j] = scol[i];
  }
  // Ey[i] of each entry is Ey[i + 1] of the one before it (a lane shift); bit
  // j of `first`: entry j of this lane starts its row (row Ey[i + 1] - 1)
  uint32_t first = 0;
#pragma unroll
  for (int j = 0; j < FR_IT; ++j) {
    const int32_t up = __shfl_up(e1[j], 1, 64);
    const int32_t e0 = lane > 0 ? up : (j > 0 ? __builtin_amdgcn_readlane(e1[j > 0 ? j - 1 : 0], 63) : ew);
    if (w0 + j * 64 + lane < n && e1[j] != e0) first |= 1u << j;
  }
  // the bitmap words as 32-bit words (sparse: the 64-bit words read
  // little-endian, word z / 32 holds bit z % 32; cold: the low halves of the
  // packed words) and the hot flags of the rows
  const uint32_t* zb32 = reinterpret_cast<const uint32_t*>(zbit);
  constexpr int ZW = MODE == FILTER_COLD ? 2 : 1;  // 32-bit words per 32 z
  uint32_t zb[FR_IT];
  int32_t h[FR_IT];
#pragma unroll
  for (int j = 0; j < FR_IT; ++j) {
    zb[j] = zb32[ZW * (z[j] >> 5)];
    h[j] = MODE == FILTER_COLD ? hot[e1[j] - 1] : 0;
  }
  uint32_t keep = 0;
  int cnt = 0;
#pragma unroll
  for (int j = 0; j < FR_IT; ++j) {
    const bool k = w0 + j * 64 + lane < n && ((zb[j] >> (z[j] & 31)) & 1u) && !h[j];
    if (k) keep |= 1u << j;
    cnt += __popcll(ballot(k));
  }
  // values of the kept entries: z itself, or its local index in the space from
  // the word's rank base (the high half, in the same cache line; a gather from
  // zsel only where the word has none)
  int32_t val[FR_IT];
#pragma unroll
  for (int j = 0; j < FR_IT; ++j) {
    if (MODE == FILTER_SPARSE) {
      val[j] = z[j];
    } else {
      val[j] = ((keep >> j) & 1u) ? int32_t(zb32[2 * (z[j] >> 5) + 1]) : 0;
    }
  }
  if (MODE == FILTER_COLD) {
#pragma unroll
    for (int j = 0; j < FR_IT; ++j) {
      if ((keep >> j) & 1u) {
        val[j] = val[j] >= 0 ? val[j] + __popc(zb[j] & ((1u << (z[j] & 31)) - 1u)) : zsel[z[j]];
      }
    }
  }
  if (lane == 0) s_wsum[wid] = cnt;
  __syncthreads();
  int32_t woff = 0, btot = 0;
#pragma unroll
  for (int w = 0; w < FR_NT / 64; ++w) {
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
  for (int j = 0; j < FR_IT; ++j) {
    const bool k = (keep >> j) & 1u;
    const uint64_t b = ballot(k);
    const int64_t before = run + __popcll(b & ltm);
    if (k) {
      out[before] = val[j];
      if (orow) orow[before] = e1[j] - 1;
    }
    if ((first >> j) & 1u) rowptr[e1[j] - 1] = int32_t(before);
    run += __popcll(b);
  }
  if (tile == ntiles - 1 && threadIdx.x == 0) {
    const int32_t t = int32_t(s_excl + btot);
    rowptr[n_rows] = t;
    *total = t;
  }
}

// space 0: the dense z, local index = dense index - first dense index of the instance
__global__ void k_zmap_dense(const int32_t* __restrict__ zflag, const int32_t* __restrict__ Edz, int64_t n_z,
                             const int32_t* __restrict__ z_base, const int32_t* __restrict__ zd_base, int n_inst,
                             int32_t* __restrict__ zmap) {
  SegCursor<int32_t> zcur(z_base, n_inst);
  zcur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(z, n_z, JP_CHUNK) {
    const int inst = zcur(int32_t(z));
    zmap[z] = zflag[z] ? Edz[z] - zd_base[inst] : -1;
  }
}

// space 1: the dense z outside the pivot row of instances with a pivot
// (rflag over the dense index, Erd its exclusive scan)
__global__ void k_zmap_resid(const int32_t* __restrict__ zflag, const int32_t* __restrict__ Edz,
                             const int32_t* __restrict__ rflag, const int32_t* __restrict__ Erd, int64_t n_z,
                             const int32_t* __restrict__ z_base, const int32_t* __restrict__ zc_base, int n_inst,
                             int32_t* __restrict__ zmap) {
  SegCursor<int32_t> zcur(z_base, n_inst);
  zcur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(z, n_z, JP_CHUNK) {
    int32_t v = -1;
    if (zflag[z]) {
      const int d = Edz[z];
      if (rflag[d]) {
        const int inst = zcur(int32_t(z));
        v = Erd[d] - zc_base[inst];
      }
    }
    zmap[z] = v;
  }
}

// pivot candidate of each instance: its hot key of rank 0 (most R rows)
__global__ void k_pivot_pick(const int32_t* __restrict__ hotrow, int64_t n_y, const int32_t* __restrict__ y_base,
                             int n_inst, int32_t* __restrict__ piv) {
  GRID_STRIDE(y, n_y) {
    if (hotrow[y] == 0) piv[n_inst == 1 ? 0 : find_inst<int32_t>(y_base, n_inst, int32_t(y))] = int32_t(y);
  }
}

// info[3i..3i+2] = (pivot, d_R(pivot), dense entries of the pivot) for instance i (pivot -1: none)
__global__ void k_pivot_info(const int32_t* __restrict__ piv, int n_inst, const int32_t* __restrict__ dR,
                             const int32_t* __restrict__ cnt_a, const int32_t* __restrict__ cnt_b,
                             int32_t* __restrict__ info) {
  GRID_STRIDE(i, n_inst) {
    const int32_t p = piv[i];
    info[3 * i] = p;
    info[3 * i + 1] = p >= 0 ? dR[p] : 0;
    info[3 * i + 2] = p >= 0 ? space_count(cnt_a, cnt_b, p) : 0;
  }
}

// inP[dense index] = 1 for every dense z of the instance's pivot row
__global__ void k_mark_pivot(const int32_t* __restrict__ Ey, const int32_t* __restrict__ scol, int64_t n,
                             const int32_t* __restrict__ y_base, int n_inst, const int32_t* __restrict__ piv,
                             const int32_t* __restrict__ zflag, const int32_t* __restrict__ Edz,
                             int32_t* __restrict__ inP) {
  SegCursor<int32_t> ycur(y_base, n_inst);
  if (chunk_first() < n) ycur.seed(Ey[chunk_first() + 1] - 1);
  CHUNK_LOOP(p, n, JP_CHUNK) {
    const int32_t y = Ey[p + 1] - 1;
    const int inst = ycur(y);
    const int32_t z = scol[p];
    if (piv[inst] == y && zflag[z]) inP[Edz[z]] = 1;
  }
}

// out[d] = 1 iff dense index d belongs to an instance with a pivot and is outside the pivot row
__global__ void k_resid_flags(const int32_t* __restrict__ inP, int64_t n, const int32_t* __restrict__ zd_base,
                              int n_inst, const int32_t* __restrict__ piv, int32_t* __restrict__ out) {
  SegCursor<int32_t> dcur(zd_base, n_inst);
  dcur.seed(int32_t(chunk_first()));
  CHUNK_LOOP(d, n, JP_CHUNK) {
    const int inst = dcur(int32_t(d));
    out[d] = (piv[inst] >= 0 && !inP[d]) ? 1 : 0;
  }
}

// flag[x] = 1 iff row x holds its instance's pivot key (one wavefront per row)
__global__ void k_row_pivot(const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol, int64_t n_x,
                            const int32_t* __restrict__ x_base, int n_inst, const int32_t* __restrict__ piv,
                            int32_t* __restrict__ flag) {
  const int lane = lane_id();
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t x = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); x < n_x; x += waves) {
    const int inst = n_inst == 1 ? 0 : find_inst<int32_t>(x_base, n_inst, int32_t(x));
    const int32_t p = piv[inst];
    bool hit = false;
    if (p >= 0) {
      for (int j = rptr[x] + lane; j < rptr[x + 1] && !hit; j += 64) hit = rcol[j] == p;
    }
    const bool any = ballot(hit) != 0;
    if (lane == 0) flag[x] = any ? 1 : 0;
  }
}

// rows with flag 1 to rows_p, the others to rows_n, both in x order
__global__ void k_split_rows(const int32_t* __restrict__ flag, const int32_t* __restrict__ E, int64_t n,
                             int32_t* __restrict__ rows_p, int32_t* __restrict__ rows_n) {
  GRID_STRIDE(x, n) {
    if (flag[x]) rows_p[E[x]] = int32_t(x);
    else rows_n[x - E[x]] = int32_t(x);
  }
}

__global__ void k_hot_list(const int32_t* __restrict__ hot, const int32_t* __restrict__ Ehot, int64_t n_y,
                           int32_t* __restrict__ hotlist) {
  GRID_STRIDE(y, n_y) {
    if (hot[y]) hotlist[Ehot[y]] = int32_t(y);
  }
}

// rank of each hot y among its instance's hot keys: more rows first, then y order
__global__ void k_hot_rank(const int32_t* __restrict__ hotlist, int64_t n_hot, const int32_t* __restrict__ Ehot,
                           const int32_t* __restrict__ y_base, int n_inst, const int32_t* __restrict__ dR,
                           int32_t* __restrict__ hotrow) {
  GRID_STRIDE(i, n_hot) {
    const int32_t y = hotlist[i];
    const int inst = n_inst == 1 ? 0 : find_inst<int32_t>(y_base, n_inst, y);
    const int lo = Ehot[y_base[inst]], hi = Ehot[y_base[inst + 1]];
    const int32_t d = dR[y];
    int rank = 0;
    for (int j = lo; j < hi; ++j) {
      const int32_t y2 = hotlist[j];
      const int32_t d2 = dR[y2];
      rank += (d2 > d || (d2 == d && y2 < y)) ? 1 : 0;
    }
    hotrow[y] = rank;
  }
}

// code of each join key (coalesced over y), then one gather per R entry
__global__ void k_key_codes(const int32_t* __restrict__ hotrow, const int32_t* __restrict__ cptr, int64_t n_y,
                            int32_t* __restrict__ ycode) {
  GRID_STRIDE(y, n_y) {
    const int32_t h = hotrow[y];
    ycode[y] = h >= 0 ? h : (cptr[y + 1] > cptr[y] ? int32_t(-2 - y) : -1);
  }
}

__global__ void k_row_codes(const int32_t* __restrict__ rcol, int64_t n, const int32_t* __restrict__ ycode,
                            int32_t* __restrict__ rcode) {
  // eight entries per thread and step: their column loads, then their code gathers, then the stores
  constexpr int U = 8;
  const int64_t c1 = chunk_first() + JP_CHUNK < n ? chunk_first() + JP_CHUNK : n;
  const int64_t step = blockDim.x;
  for (int64_t j0 = chunk_first() + threadIdx.x; j0 < c1; j0 += U * step) {
    int32_t y[U], v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) y[u] = rcol[j0 + u * step < c1 ? j0 + u * step : c1 - 1];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ycode[y[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j0 + u * step < c1) rcode[j0 + u * step] = v[u];
  }
}

// every table slot is written exactly once: by the first entry of y at or
// after the window start (entries), or by the row end (tail)
__global__ void k_cold_win_entries(const int32_t* __restrict__ cptr, const int32_t* __restrict__ ccol,
                                   const int32_t* __restrict__ crow, int64_t n_cold,
                                   const int32_t* __restrict__ y_base, int n_inst, const int64_t* __restrict__ cw_off,
                                   int32_t* __restrict__ cw) {
  // crow[p] = row of entry p; four entries per thread and step, loads first
  SegCursor<int32_t> ycur(y_base, n_inst);
  ycur.seed(crow[chunk_first() < n_cold ? chunk_first() : n_cold - 1]);
  const int64_t c1 = chunk_first() + JP_CHUNK < n_cold ? chunk_first() + JP_CHUNK : n_cold;
  const int64_t step = blockDim.x;
  for (int64_t p0 = chunk_first() + threadIdx.x; p0 < c1; p0 += 4 * step) {
    int32_t y[4], d[4], dp[4], a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step < c1 ? p0 + u * step : c1 - 1;
      y[u] = crow[p];
      d[u] = ccol[p];
      dp[u] = ccol[p > 0 ? p - 1 : 0];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = cptr[y[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step;
      if (p >= c1) break;
      const int inst = ycur(y[u]);
      const int ny = y_base[inst + 1] - y_base[inst];
      const int yl = y[u] - y_base[inst];
      const int wp = d[u] / DW_BITS;
      const int wprev = p == a[u] ? -1 : dp[u] / DW_BITS;
      int32_t* t = cw + cw_off[inst] + yl;
      for (int w = wprev + 1; w <= wp; ++w) t[int64_t(w) * ny] = int32_t(p);
    }
  }
}

__global__ void k_cold_win_tail(const int32_t* __restrict__ cptr, const int32_t* __restrict__ ccol, int64_t n_y,
                                const int32_t* __restrict__ y_base, const int32_t* __restrict__ zd_base, int n_inst,
                                const int64_t* __restrict__ cw_off, int32_t* __restrict__ cw) {
  // one row per thread; the instance cursor is seeded once per wave
  SegCursor<int32_t> ycur(y_base, n_inst);
  const int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t y0 = y - lane_id();  // the wave's first row
  ycur.seed(int32_t(y0 < n_y ? y0 : 0));
  if (y < n_y) {
    const int inst = ycur(int32_t(y));
    const int zd = zd_base[inst + 1] - zd_base[inst];
    if (zd <= 0) return;
    const int nwin = (zd + DW_BITS - 1) / DW_BITS;
    const int ny = y_base[inst + 1] - y_base[inst];
    const int yl = int(y) - y_base[inst];
    const int a = cptr[y], b = cptr[y + 1];
    const int wlast = b > a ? ccol[b - 1] / DW_BITS : -1;
    int32_t* t = cw + cw_off[inst] + yl;
    for (int w = wlast + 1; w <= nwin; ++w) t[int64_t(w) * ny] = b;
  }
}

// window-major layout of the cold entries: segment counts per (window, y)
__global__ void k_cold_win_counts(const int32_t* __restrict__ cw, const int64_t* __restrict__ cw_off,
                                  const int64_t* __restrict__ cwm_off, const int32_t* __restrict__ y_base,
                                  const int32_t* __restrict__ zd_base, int n_inst, int64_t n_y,
                                  int32_t* __restrict__ cnt) {
  // one row per thread (a row walks all windows of its instance); the
  // instance cursor is seeded once per wave instead of a search per row
  SegCursor<int32_t> ycur(y_base, n_inst);
  const int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t y0 = y - lane_id();  // the wave's first row
  ycur.seed(int32_t(y0 < n_y ? y0 : 0));
  if (y < n_y) {
    const int inst = ycur(int32_t(y));
    const int zd = zd_base[inst + 1] - zd_base[inst];
    if (zd <= 0) return;
    const int nwin = (zd + DW_BITS - 1) / DW_BITS;
    const int ny = y_base[inst + 1] - y_base[inst];
    const int yl = int(y) - y_base[inst];
    const int32_t* t = cw + cw_off[inst] + yl;
    int32_t* o = cnt + cwm_off[inst] + yl;
    for (int w = 0; w < nwin; ++w) o[int64_t(w) * ny] = t[int64_t(w + 1) * ny] - t[int64_t(w) * ny];
  }
}

__global__ void k_cold_win_scatter(const int32_t* __restrict__ ccol, const int32_t* __restrict__ crow,
                                   int64_t n_cold, const int32_t* __restrict__ y_base, int n_inst,
                                   const int32_t* __restrict__ cw, const int64_t* __restrict__ cw_off,
                                   const int32_t* __restrict__ wptr, const int64_t* __restrict__ cwm_off,
                                   int32_t* __restrict__ ccol_w) {
  // crow[p] = row of entry p; four entries per thread and step, loads first
  SegCursor<int32_t> ycur(y_base, n_inst);
  ycur.seed(crow[chunk_first() < n_cold ? chunk_first() : n_cold - 1]);
  const int64_t c1 = chunk_first() + JP_CHUNK < n_cold ? chunk_first() + JP_CHUNK : n_cold;
  const int64_t step = blockDim.x;
  for (int64_t p0 = chunk_first() + threadIdx.x; p0 < c1; p0 += 4 * step) {
    int32_t y[4], d[4], inst[4], b0[4], e0[4];
    int64_t slot[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step < c1 ? p0 + u * step : c1 - 1;
      y[u] = crow[p];
      d[u] = ccol[p];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      inst[u] = ycur(y[u]);
      const int ny = y_base[inst[u] + 1] - y_base[inst[u]];
      slot[u] = int64_t(d[u] / DW_BITS) * ny + (y[u] - y_base[inst[u]]);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      b0[u] = wptr[cwm_off[inst[u]] + slot[u]];
      e0[u] = cw[cw_off[inst[u]] + slot[u]];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t p = p0 + u * step;
      if (p < c1) ccol_w[b0[u] + (p - e0[u])] = d[u];
    }
  }
}

}  // namespace

void cold_window_major(const int32_t* ccol, const int32_t* crow, int64_t n_y, int64_t n_cold, const int32_t* y_base,
                       const int32_t* zd_base, int n_inst, const int32_t* cw, const int64_t* cw_off,
                       const int64_t* cwm_off, int64_t cwm_total, int32_t* wptr, int32_t* ccol_w, hipStream_t s,
                       Arena& a) {
  int32_t* cnt = a.alloc<int32_t>(std::max<int64_t>(cwm_total, 1), s);
  if (n_y > 0)
    hipLaunchKernelGGL(k_cold_win_counts, dim3(chunk_grid(n_y, NT)), dim3(NT), 0, s, cw, cw_off, cwm_off, y_base,
                       zd_base, n_inst, n_y, cnt);
  JP_LAUNCH_CHECK();
  scan_excl_i32(cnt, wptr, cwm_total, s, a);
  if (n_cold > 0)
    hipLaunchKernelGGL(k_cold_win_scatter, dim3(chunk_grid(n_cold)), dim3(NT), 0, s, ccol, crow, n_cold, y_base,
                       n_inst, cw, cw_off, wptr, cwm_off, ccol_w);
  JP_LAUNCH_CHECK();
  a.give_back(cnt, s);
}

void dense_flags(const int32_t* m_z, int64_t n_z, const int32_t* z_base, int n_inst, const int64_t* tau, int32_t* flag,
                 hipStream_t s) {
  if (n_z <= 0) return;
  hipLaunchKernelGGL(k_dense_flags, dim3(chunk_grid(n_z)), dim3(NT), 0, s, m_z, n_z, z_base, n_inst, tau, flag);
  JP_LAUNCH_CHECK();
}

void dense_index(const int32_t* flag, const int32_t* Edz, int64_t n_z, int32_t* dz2z, hipStream_t s) {
  if (n_z <= 0) return;
  hipLaunchKernelGGL(k_dense_index, dim3(grid(n_z)), dim3(NT), 0, s, flag, Edz, n_z, dz2z);
  JP_LAUNCH_CHECK();
}

void filter_rows(bool cold, const int32_t* Ey, const int32_t* scol, int64_t n, const int32_t* zsel, int64_t n_z,
                 const int32_t* hot, int32_t* out, int32_t* out_row, int32_t* rowptr, int64_t n_rows, int32_t* total,
                 hipStream_t s, Arena& a) {
  if (n <= 0) {
    fill_i32(rowptr, n_rows + 1, 0, s);
    fill_i32(total, 1, 0, s);
    return;
  }
  const int64_t nw = cold ? (n_z + 31) / 32 : (n_z + 63) / 64;  // cold: packed 32-bit words with rank bases
  uint64_t* zbit = a.alloc<uint64_t>(std::max<int64_t>(nw, 1), s);
  const int gb = int(std::min<int64_t>((n_z + NT - 1) / NT, 1 << 16));
  if (cold) hipLaunchKernelGGL(k_filter_bits<FILTER_COLD>, dim3(gb > 0 ? gb : 1), dim3(NT), 0, s, zsel, n_z, zbit);
  else hipLaunchKernelGGL(k_filter_bits<FILTER_SPARSE>, dim3(gb > 0 ? gb : 1), dim3(NT), 0, s, zsel, n_z, zbit);
  const int64_t nt = (n + FR_TILE - 1) / FR_TILE;
  uint64_t* status = a.alloc<uint64_t>(nt + 2, s);
  fill_i64(reinterpret_cast<int64_t*>(status), nt + 2, 0, s);
  if (cold)
    hipLaunchKernelGGL(k_filter_rows<FILTER_COLD>, dim3(int(nt)), dim3(FR_NT), 0, s, Ey, scol, n, zsel,
                       (const uint64_t*)zbit, hot, out, out_row, rowptr, n_rows, total, status, nt);
  else
    hipLaunchKernelGGL(k_filter_rows<FILTER_SPARSE>, dim3(int(nt)), dim3(FR_NT), 0, s, Ey, scol, n, zsel,
                       (const uint64_t*)zbit, hot, out, out_row, rowptr, n_rows, total, status, nt);
  JP_LAUNCH_CHECK();
  a.give_back(status, s);
  a.give_back(zbit, s);
}

void remap_rowptr(const int32_t* rowptr, const int32_t* E, int64_t n_y, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_remap_rowptr, dim3(grid(n_y + 1)), dim3(NT), 0, s, rowptr, E, n_y, out);
  JP_LAUNCH_CHECK();
}

void hot_histogram(const int32_t* cnt_a, const int32_t* cnt_b, const int32_t* dR, int64_t n_y,
                   const int32_t* y_base, int n_inst, int32_t* hist, hipStream_t s) {
  fill_i32(hist, int64_t(n_inst) * 32, 0, s);
  if (n_y <= 0) return;
  hipLaunchKernelGGL(k_hot_histogram, dim3(chunk_grid(n_y)), dim3(NT), 0, s, cnt_a, cnt_b, dR, n_y, y_base, n_inst,
                     hist);
  JP_LAUNCH_CHECK();
}

void hot_flags(const int32_t* cnt_a, const int32_t* cnt_b, const int32_t* dR, int64_t n_y, const int32_t* y_base,
               int n_inst, const int64_t* theta, int32_t* hot, hipStream_t s) {
  if (n_y <= 0) return;
  hipLaunchKernelGGL(k_hot_flags, dim3(chunk_grid(n_y)), dim3(NT), 0, s, cnt_a, cnt_b, dR, n_y, y_base, n_inst, theta, hot);
  JP_LAUNCH_CHECK();
}

void build_hot_bits(const int32_t* hotlist, int64_t n_hot, const int32_t* sptr, const int32_t* scol, int64_t n_s,
                    const int32_t* hotrow, const int32_t* y_base, const int32_t* zmap, const int64_t* hb_off,
                    const int32_t* row_words, int n_inst, uint32_t* hb, hipStream_t s, Arena& a) {
  if (n_hot <= 0 || n_s <= 0) return;
  int32_t* len = a.alloc<int32_t>(n_hot, s);
  int32_t* hoff = a.alloc<int32_t>(n_hot + 1, s);
  int32_t* pdel = a.alloc<int32_t>(n_hot, s);
  int64_t* rbase = a.alloc<int64_t>(n_hot, s);
  hipLaunchKernelGGL(k_hot_row_lengths, dim3(grid(n_hot)), dim3(NT), 0, s, hotlist, n_hot, sptr, len);
  JP_LAUNCH_CHECK();
  scan_excl_i32(len, hoff, n_hot, s, a);
  hipLaunchKernelGGL(k_hot_row_info, dim3(grid(n_hot)), dim3(NT), 0, s, hotlist, n_hot, hoff, sptr, hotrow, y_base,
                     n_inst, hb_off, row_words, pdel, rbase);
  JP_LAUNCH_CHECK();
  // the hot rows hold at most all n_s entries; enough blocks to fill the chip,
  // each striding over chunks of the concatenated rows
  const int blocks = std::min(chunk_grid(n_s), 2048);
  hipLaunchKernelGGL(k_build_hot_bits, dim3(blocks), dim3(NT), 0, s, hoff, int(n_hot), pdel, rbase, scol, zmap, hb);
  JP_LAUNCH_CHECK();
  a.give_back(rbase, s);
  a.give_back(pdel, s);
  a.give_back(hoff, s);
  a.give_back(len, s);
}

void space_flags(const int32_t* scol, int64_t n, const int32_t* zmap, int32_t* flag, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_space_flags, dim3(grid(n)), dim3(NT), 0, s, scol, n, zmap, flag);
  JP_LAUNCH_CHECK();
}

void zmap_dense(const int32_t* zflag, const int32_t* Edz, int64_t n_z, const int32_t* z_base, const int32_t* zd_base,
                int n_inst, int32_t* zmap, hipStream_t s) {
  if (n_z <= 0) return;
  hipLaunchKernelGGL(k_zmap_dense, dim3(chunk_grid(n_z)), dim3(NT), 0, s, zflag, Edz, n_z, z_base, zd_base, n_inst, zmap);
  JP_LAUNCH_CHECK();
}

void zmap_resid(const int32_t* zflag, const int32_t* Edz, const int32_t* rflag, const int32_t* Erd, int64_t n_z,
                const int32_t* z_base, const int32_t* zc_base, int n_inst, int32_t* zmap, hipStream_t s) {
  if (n_z <= 0) return;
  hipLaunchKernelGGL(k_zmap_resid, dim3(chunk_grid(n_z)), dim3(NT), 0, s, zflag, Edz, rflag, Erd, n_z, z_base, zc_base,
                     n_inst, zmap);
  JP_LAUNCH_CHECK();
}

void pivot_info(const int32_t* hotrow, int64_t n_y, const int32_t* y_base, int n_inst, const int32_t* dR,
                const int32_t* cnt_a, const int32_t* cnt_b, int32_t* piv, int32_t* info, hipStream_t s) {
  fill_i32(piv, n_inst, -1, s);
  if (n_y > 0) {
    hipLaunchKernelGGL(k_pivot_pick, dim3(grid(n_y)), dim3(NT), 0, s, hotrow, n_y, y_base, n_inst, piv);
    JP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_pivot_info, dim3(grid(n_inst)), dim3(NT), 0, s, piv, n_inst, dR, cnt_a, cnt_b, info);
  JP_LAUNCH_CHECK();
}

void mark_pivot(const int32_t* Ey, const int32_t* scol, int64_t n, const int32_t* y_base, int n_inst,
                const int32_t* piv, const int32_t* zflag, const int32_t* Edz, int32_t* inP, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mark_pivot, dim3(chunk_grid(n)), dim3(NT), 0, s, Ey, scol, n, y_base, n_inst, piv, zflag, Edz, inP);
  JP_LAUNCH_CHECK();
}

void resid_flags(const int32_t* inP, int64_t n, const int32_t* zd_base, int n_inst, const int32_t* piv, int32_t* out,
                 hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_resid_flags, dim3(chunk_grid(n)), dim3(NT), 0, s, inP, n, zd_base, n_inst, piv, out);
  JP_LAUNCH_CHECK();
}

void row_pivot_flags(const int32_t* rptr, const int32_t* rcol, int64_t n_x, const int32_t* x_base, int n_inst,
                     const int32_t* piv, int32_t* flag, hipStream_t s) {
  if (n_x <= 0) return;
  hipLaunchKernelGGL(k_row_pivot, dim3(grid(n_x * 64, 1 << 16)), dim3(NT), 0, s, rptr, rcol, n_x, x_base, n_inst, piv,
                     flag);
  JP_LAUNCH_CHECK();
}

void split_rows(const int32_t* flag, const int32_t* E, int64_t n, int32_t* rows_p, int32_t* rows_n, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_split_rows, dim3(grid(n)), dim3(NT), 0, s, flag, E, n, rows_p, rows_n);
  JP_LAUNCH_CHECK();
}

void hot_rank(const int32_t* hot, const int32_t* Ehot, int64_t n_y, int64_t n_hot, const int32_t* y_base, int n_inst,
              const int32_t* dR, int32_t* hotlist, int32_t* hotrow, hipStream_t s) {
  fill_i32(hotrow, n_y, -1, s);
  if (n_y <= 0 || n_hot <= 0) return;
  hipLaunchKernelGGL(k_hot_list, dim3(grid(n_y)), dim3(NT), 0, s, hot, Ehot, n_y, hotlist);
  JP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_hot_rank, dim3(grid(n_hot)), dim3(NT), 0, s, hotlist, n_hot, Ehot, y_base, n_inst, dR, hotrow);
  JP_LAUNCH_CHECK();
}

void row_codes(const int32_t* rcol, int64_t n, const int32_t* hotrow, const int32_t* cptr, int64_t n_y,
               int32_t* ycode, int32_t* rcode, hipStream_t s) {
  if (n <= 0 || n_y <= 0) return;
  hipLaunchKernelGGL(k_key_codes, dim3(grid(n_y)), dim3(NT), 0, s, hotrow, cptr, n_y, ycode);
  JP_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_row_codes, dim3(chunk_grid(n)), dim3(NT), 0, s, rcol, n, ycode, rcode);
  JP_LAUNCH_CHECK();
}

void cold_windows(const int32_t* cptr, const int32_t* ccol, const int32_t* crow, int64_t n_y, int64_t n_cold,
                  const int32_t* y_base, const int32_t* zd_base, int n_inst, const int64_t* cw_off, int32_t* cw,
                  hipStream_t s) {
  if (n_y <= 0) return;
  if (n_cold > 0) {
    hipLaunchKernelGGL(k_cold_win_entries, dim3(chunk_grid(n_cold)), dim3(NT), 0, s, cptr, ccol, crow, n_cold, y_base,
                       n_inst, cw_off, cw);
    JP_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_cold_win_tail, dim3(chunk_grid(n_y, NT)), dim3(NT), 0, s, cptr, ccol, n_y, y_base, zd_base,
                     n_inst, cw_off, cw);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
