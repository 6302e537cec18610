// DenseEC (paper Sec. 2.5, Alg. 3) for the dense z's of the partition:
// C[x, z] = OR over y of R[x, y] AND S[y, z].
//
// The paper tests one (x, z) pair at a time, either by a SIMD AND of the two
// |Y|-bit bitmaps or by probing Bitmap_z at each y of x, stopping at the
// first hit.  Here one wavefront builds a whole window of an x row at once:
// the row's "hot" join keys (y with many dense S entries) are kept as bit rows
// over the dense z index and are ORed word by word (32 z per lane-op), and the
// remaining "cold" keys are scattered from their z-sorted CSR rows into an
// LDS copy of the window.  The window is then popcounted (count mode) or
// written out in z order (write mode).
//
// A workgroup owns 128 consecutive rows and a group of consecutive windows;
// the grid is ordered window-group-major, so the workgroups resident at one
// time all read the same few windows of the hot rows and of the cold table,
// which then stay in each XCD's L2 instead of streaming from HBM.  The
// window slices of the T_STAGE hot keys shared by the most rows are staged in
// LDS once per window for all 128 rows; rarer hot keys are read from the
// caches.  Per-entry codes (hot rank / cold key) stay in registers across the
// windows, and the cold entries are stored window-major with per-(window, key)
// segment bounds, so the 64 lanes of a wave split a row's cold entries evenly
// and one window's cold data is a compact, cache-resident range.
#include <cstdlib>

#include "common.h"
#include "prim.h"
#include "stages.h"
#include "../../include/jp.h"

namespace jp {
namespace {

constexpr int NT = 1024;                  // 16 waves share one LDS stage (8 waves per SIMD)
constexpr int WAVES = NT / 64;
constexpr int RPW = 8;                    // rows per wavefront
constexpr int RB = WAVES * RPW;           // rows per workgroup
constexpr int WPL = DW_WORDS / 64;        // words of a window per lane
constexpr int Q = WPL / 4;                // uint4 per lane
constexpr int QW = DW_WORDS / 4;          // uint4 per window slice

// LDS operations of one wavefront execute in issue order, so ordering the
// row buffer's stores, atomics and loads across lanes only needs the
// compiler not to move them past each other.
__device__ __forceinline__ void lds_fence() { __builtin_amdgcn_wave_barrier(); }

// uint4 columns (64 lanes x 4 words = 256 words each) of the window starting
// at z index wstart that hold dense z of a range of zd dense z (wstart < zd)
__device__ __forceinline__ int win_cols(int zd, int32_t wstart) {
  const int words = min(DW_WORDS, (zd - wstart + 31) / 32);
  return (words + 255) / 256;
}

__device__ __forceinline__ int popc4(uint4 v) { return __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w); }

__device__ __forceinline__ void or4(uint4& a, const uint4 b) {
  a.x |= b.x;
  a.y |= b.y;
  a.z |= b.z;
  a.w |= b.w;
}

// ORs the hot keys among one wave's 64 codes into acc (LDS-staged or cached)
template <int QN>
__device__ __forceinline__ void hot_or(uint4 (&acc)[QN], int code, bool staged, int t_eff,
                                       const uint4 (*stage)[QW], const uint32_t* hbase, int64_t rw) {
  const int lane = lane_id();
  uint64_t hm = ballot(code >= 0);
  // staged keys: LDS reads
  const uint64_t sm = ballot(code >= 0 && staged && code < t_eff);
  uint64_t m = sm;
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int k = __builtin_amdgcn_readlane(code, l);
#pragma unroll
    for (int q = 0; q < QN; ++q) or4(acc[q], stage[k][q * 64 + lane]);
  }
  // other hot keys: cached global reads
  m = hm & ~sm;
  while (m) {
    const int l0 = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int k0 = __builtin_amdgcn_readlane(code, l0);
    const uint4* s0 = reinterpret_cast<const uint4*>(hbase + int64_t(k0) * rw);
#pragma unroll
    for (int q = 0; q < QN; ++q) or4(acc[q], s0[q * 64 + lane]);
  }
}

// hot_or over the first qa of the QN uint4 columns only (a window that the
// dense range ends inside: the other columns hold padding words)
template <int QN>
__device__ __forceinline__ void hot_or_part(uint4 (&acc)[QN], int code, bool staged, int t_eff,
                                            const uint4 (*stage)[QW], const uint32_t* hbase, int64_t rw, int qa) {
  const int lane = lane_id();
  uint64_t hm = ballot(code >= 0);
  const uint64_t sm = ballot(code >= 0 && staged && code < t_eff);
  uint64_t m = sm;
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int k = __builtin_amdgcn_readlane(code, l);
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (q < qa) or4(acc[q], stage[k][q * 64 + lane]);
  }
  m = hm & ~sm;
  while (m) {
    const int l0 = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int k0 = __builtin_amdgcn_readlane(code, l0);
    const uint4* s0 = reinterpret_cast<const uint4*>(hbase + int64_t(k0) * rw);
#pragma unroll
    for (int q = 0; q < QN; ++q)
      if (q < qa) or4(acc[q], s0[q * 64 + lane]);
  }
}

// scatters the cold entries of one wave's segments (lane = one key) into the
// LDS window of the row: one segment at a time, its entries spread over the
// lanes (segment bounds are wave-uniform scalars)
__device__ __forceinline__ void cold_scatter(int s0, int len, const int32_t* __restrict__ ccol, int32_t wstart,
                                             uint32_t* rowbuf) {
  const int lane = lane_id();
  uint64_t m = ballot(len > 0);
  while (m) {
    const int l = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int ss = __builtin_amdgcn_readlane(s0, l);
    const int ll = __builtin_amdgcn_readlane(len, l);
    const int32_t* src = ccol + ss;
    for (int t = lane; t < ll; t += 64) {
      const int dl = src[t] - wstart;
      atomicOr(&rowbuf[dl >> 5], 1u << (dl & 31));
    }
  }
}

// Rows are slots [0, n_rows): slot i is row rows[i] (a list, count mode), the
// i-th row of the instances listed by seg_base / seg_x0 (first x of each,
// running row count), or x_lo + i.  In count mode the row's count starts at base_cnt[instance] (the
// pivot row's size when the rows are evaluated outside the pivot's z) and is
// stored, or added when the grid has several window groups or `accumulate`.
template <bool WRITE>
__global__ void __launch_bounds__(NT, 8) k_dense_bits(RowCtx c, int64_t x_lo, int64_t n_rows,
                                                   const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ seg_base,
                                                   const int32_t* __restrict__ seg_x0, int seg_m,
                                                   const int32_t* __restrict__ base_cnt, int accumulate, int wgroup,
                                                   int skip_narrow, int32_t* __restrict__ cnt,
                                                   const int64_t* __restrict__ off, int32_t* __restrict__ out,
                                                   int64_t out_n) {
  __shared__ uint4 stage[T_STAGE][QW];
  __shared__ uint4 rowbuf_all[WAVES][QW];
  __shared__ int s_maxwin[WAVES];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  uint32_t* rowbuf = reinterpret_cast<uint32_t*>(rowbuf_all[wid]);
  uint4* rowbuf4 = rowbuf_all[wid];

  const int64_t rb0 = int64_t(blockIdx.x) * RB;  // first slot of the block
  const int64_t r0 = rb0 + int64_t(wid) * RPW;
  const int nrows = r0 >= n_rows ? 0 : int((n_rows - r0) < RPW ? (n_rows - r0) : RPW);
  const int64_t base_off = WRITE ? off[x_lo] : 0;

  // slot -> row (slots ascend with rows inside a block)
  SegCursor<int32_t> scur(seg_base, seg_m);
  if (seg_base) scur.seed(int32_t(rb0));
  auto row_of = [&](int64_t slot) -> int64_t {
    if (rows) return rows[slot];
    if (seg_base) {
      const int sg = scur(int32_t(slot));
      return int64_t(seg_x0[sg]) + (slot - scur.lo);
    }
    return x_lo + slot;
  };
  // instance of the block's first row: its hottest keys are staged in LDS
  const int64_t xb0 = row_of(rb0);
  SegCursor<int32_t> icur(c.x_base, c.n_inst);
  icur.seed(int32_t(xb0));
  const int inst0 = icur.cur;
  const int zd0 = c.zd_base[inst0 + 1] - c.zd_base[inst0];
  // rows of instances with at most NARROW_MAX dense z are left to k_dense_narrow
  const int nwin0 = (skip_narrow && zd0 <= NARROW_MAX) ? 0 : (zd0 + DW_BITS - 1) / DW_BITS;
  const int k0 = c.Ehot[c.y_base[inst0 + 1]] - c.Ehot[c.y_base[inst0]];
  const int t_eff = k0 < T_STAGE ? k0 : T_STAGE;
  const uint32_t* hb0 = c.hb + c.hb_off[inst0];
  const int64_t rw0 = c.row_words[inst0];

  // lane r < nrows describes row r0 + r
  int my_inst = 0, my_nwin = 0, my_a = 0, my_b = 0;
  int64_t my_x = 0;
  int64_t my_acc = 0;  // count (count mode) or write position (write mode)
  if (lane < nrows) {
    const int64_t x = row_of(r0 + lane);
    my_x = x;
    my_inst = icur(int32_t(x));
    const int zd = c.zd_base[my_inst + 1] - c.zd_base[my_inst];
    my_nwin = (skip_narrow && zd <= NARROW_MAX) ? 0 : (zd + DW_BITS - 1) / DW_BITS;
    my_a = c.rptr[x];
    my_b = c.rptr[x + 1];
    if (WRITE) my_acc = off[x] - base_off;
    else if (base_cnt && blockIdx.y == 0) my_acc = base_cnt[my_inst];
  }
  // the first 64 codes of every row stay in registers for all windows
  int code[RPW];
#pragma unroll
  for (int r = 0; r < RPW; ++r) {
    const int a = __builtin_amdgcn_readlane(my_a, r), b = __builtin_amdgcn_readlane(my_b, r);
    code[r] = (r < nrows && a + lane < b) ? c.rcode[a + lane] : -1;
  }
  const int wmax = wave_max(my_nwin);
  if (lane == 0) s_maxwin[wid] = wmax;
  __syncthreads();
  int maxwin = 0;
#pragma unroll
  for (int i = 0; i < WAVES; ++i) maxwin = s_maxwin[i] > maxwin ? s_maxwin[i] : maxwin;

  const int w_lo = int(blockIdx.y) * wgroup;
  const int w_hi = maxwin < w_lo + wgroup ? maxwin : w_lo + wgroup;
  for (int w = w_lo; w < w_hi; ++w) {
    const int32_t wstart = w * DW_BITS;
    __syncthreads();
    if (w < nwin0) {
      // only the uint4 columns that hold dense z of the first instance
      const int qw0 = win_cols(zd0, wstart) * 64;
      for (int i = threadIdx.x; i < t_eff * qw0; i += NT) {
        const int k = i / qw0, q = i - k * qw0;
        stage[k][q] = reinterpret_cast<const uint4*>(hb0 + int64_t(k) * rw0 + int64_t(w) * DW_WORDS)[q];
      }
    }
    __syncthreads();

    // the rows' first codes shift through cr, so the row loop stays rolled
    // (unrolled, its scalar state spills)
    int cr[RPW];
#pragma unroll
    for (int k = 0; k < RPW; ++k) cr[k] = code[k];
#pragma unroll 1
    for (int r = 0; r < nrows; ++r) {
      const int cd_r = cr[0];
#pragma unroll
      for (int k = 0; k + 1 < RPW; ++k) cr[k] = cr[k + 1];
      const int nwin_r = __builtin_amdgcn_readlane(my_nwin, r);
      if (w >= nwin_r) continue;
      const int inst = __builtin_amdgcn_readlane(my_inst, r);
      const int a = __builtin_amdgcn_readlane(my_a, r), b = __builtin_amdgcn_readlane(my_b, r);
      const bool staged = inst == inst0;
      const uint32_t* hbase = c.hb + c.hb_off[inst] + int64_t(w) * DW_WORDS;
      const int64_t rw = c.row_words[inst];
      const int yb = c.y_base[inst];
      const int ny = c.y_base[inst + 1] - yb;
      const int32_t* wp = c.wptr + c.cwm_off[inst] + int64_t(w) * ny;
      // uint4 columns of this window that hold dense z of the row's instance
      const int qa = win_cols(c.zd_base[inst + 1] - c.zd_base[inst], wstart);

      // bounds of this window's cold segments: issued first, used after the hot ORs
      const int cd = cd_r;
      int s0 = 0, len = 0;
      if (cd <= -2) {
        const int yl = (-2 - cd) - yb;
        s0 = wp[yl];
        len = wp[yl + 1] - s0;
      }
      bool any_cold = ballot(cd <= -2) != 0;

      uint4 acc[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) acc[q] = make_uint4(0, 0, 0, 0);
      if (qa == Q) {
        hot_or<Q>(acc, cd, staged, t_eff, stage, hbase, rw);
        for (int c0 = a + 64; c0 < b; c0 += 64) {  // rows with more than 64 join keys
          const int j = c0 + lane;
          const int cx = j < b ? c.rcode[j] : -1;
          any_cold |= ballot(cx <= -2) != 0;
          hot_or<Q>(acc, cx, staged, t_eff, stage, hbase, rw);
        }
      } else {
        hot_or_part<Q>(acc, cd, staged, t_eff, stage, hbase, rw, qa);
        for (int c0 = a + 64; c0 < b; c0 += 64) {
          const int j = c0 + lane;
          const int cx = j < b ? c.rcode[j] : -1;
          any_cold |= ballot(cx <= -2) != 0;
          hot_or_part<Q>(acc, cx, staged, t_eff, stage, hbase, rw, qa);
        }
      }
      if (any_cold) {
        // columns past qa stay zero in acc (cold z lie in the dense range)
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (q < qa) rowbuf4[q * 64 + lane] = acc[q];
        lds_fence();
        cold_scatter(s0, len, c.ccol, wstart, rowbuf);
        for (int c0 = a + 64; c0 < b; c0 += 64) {
          const int j = c0 + lane;
          const int cx = j < b ? c.rcode[j] : -1;
          int t0 = 0, tl = 0;
          if (cx <= -2) {
            const int yl = (-2 - cx) - yb;
            t0 = wp[yl];
            tl = wp[yl + 1] - t0;
          }
          cold_scatter(t0, tl, c.ccol, wstart, rowbuf);
        }
        lds_fence();
#pragma unroll
        for (int q = 0; q < Q; ++q)
          if (q < qa) acc[q] = rowbuf4[q * 64 + lane];
        lds_fence();
      }

      if (!WRITE) {
        int pc = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) pc += popc4(acc[q]);
        const int tot = wave_sum_dpp(pc);
        if (lane == r) my_acc += tot;
      } else {
        const int64_t pos0 = __shfl(my_acc, r, 64);
        int64_t qbase = 0;
        const int32_t dzb = c.zd_base[inst];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int pc = popc4(acc[q]);
          const int incl = wave_incl_scan(pc);
          const int tq = __shfl(incl, 63, 64);
          int64_t pos = pos0 + qbase + (incl - pc);
          const uint32_t wv[4] = {acc[q].x, acc[q].y, acc[q].z, acc[q].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            uint32_t word = wv[e];
            const int32_t wbase = wstart + (q * 256 + lane * 4 + e) * 32;
            while (word) {
              const int bit = __ffs(word) - 1;
              word &= word - 1;
              if (pos < out_n) out[pos] = c.dz2z[dzb + wbase + bit];  // out_n bounds a stale count
              ++pos;
            }
          }
          qbase += tq;
        }
        if (lane == r) my_acc += qbase;
      }
    }
  }
  if (!WRITE && lane < nrows) {
    if (gridDim.y == 1 && !accumulate) cnt[my_x] = int32_t(my_acc);
    else if (my_acc) atomicAdd(&cnt[my_x], int32_t(my_acc));
  }
}

// Count mode for rows of instances with few dense z (0 < Z_d <= 32 * LANES * WPL):
// the whole dense range is one short bit row, so a group of LANES lanes owns
// a row, WPL 32-z words per lane, and a wave counts 64 / LANES rows at once
// (each row is a chain of dependent loads, so more rows per wave keep more
// loads in flight)
// (the window kernel would spend a 32768-z window, 1024 words, on each).  The
// groups walk their rows' join keys LANES at a time: hot keys are ORed one
// per group per step (each group loads its own key's words), cold keys are
// scattered into the group's LDS words.  Slot i is row rows[i] (a list: rows
// of other instances are skipped), or the i-th row of the class's narrow
// instances (c.nar_x0 / c.nar_base of class CLS).
template <int LANES, int WPL>
__global__ void __launch_bounds__(256) k_dense_narrow(RowCtx c, int64_t n_slots, const int32_t* __restrict__ rows,
                                                   int accumulate, int32_t* __restrict__ cnt) {
  static_assert(WPL == 1 || WPL == 2 || WPL == 4 || WPL == 8, "a word, a uint2, a uint4 or two uint4 per lane");
  constexpr int GROUPS = 64 / LANES;
  constexpr int ZMAX = 32 * LANES * WPL;
  constexpr int CLS = ZMAX == NARROW_SMALL ? 0 : ZMAX == NARROW_MID ? 1 : 2;
  constexpr int ZMIN = CLS == 0 ? 1 : CLS == 1 ? NARROW_SMALL + 1 : NARROW_MID + 1;
  static_assert(ZMAX == (CLS == 0 ? NARROW_SMALL : CLS == 1 ? NARROW_MID : NARROW_MAX), "class bounds");
  __shared__ uint32_t buf_all[4][64 * WPL];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  const int grp = lane / LANES, gl = lane % LANES;
  uint32_t* buf = &buf_all[wid][grp * LANES * WPL];
#pragma unroll
  for (int e = 0; e < WPL; ++e) buf[gl * WPL + e] = 0u;
  lds_fence();

  const int64_t slot0 = (int64_t(blockIdx.x) * 4 + wid) * GROUPS;
  const int64_t slot = slot0 + grp;
  const bool valid = slot < n_slots;
  int64_t x = 0;
  int32_t x_first = 0;  // the wave's first row (rows ascend with the slots): seeds the instance cursor
  if (rows) {
    x = valid ? int64_t(rows[slot]) : 0;
    x_first = slot0 < n_slots ? rows[slot0] : 0;
  } else {
    SegCursor<int32_t> scur(c.nar_base[CLS], c.nar_m[CLS]);
    scur.seed(int32_t(slot0 < n_slots ? slot0 : 0));
    if (valid) {
      const int sg = scur(int32_t(slot));
      x = int64_t(c.nar_x0[CLS][sg]) + (slot - scur.lo);
    }
    x_first = __shfl(int32_t(x), 0, 64);
  }
  SegCursor<int32_t> icur(c.x_base, c.n_inst);
  icur.seed(x_first);
  const int inst = valid ? icur(int32_t(x)) : 0;
  const int zd = c.zd_base[inst + 1] - c.zd_base[inst];
  const bool active = valid && zd >= ZMIN && zd <= ZMAX;
  if (!__ballot(active)) return;
  const int nwords = (zd + 31) >> 5;
  int a = 0, b = 0;
  if (active) {
    a = c.rptr[x];
    b = c.rptr[x + 1];
  }
  const uint32_t* hrow = c.hb + c.hb_off[inst];
  const int64_t rw = c.row_words[inst];
  const int yb = c.y_base[inst];
  const int32_t* wp = c.wptr + c.cwm_off[inst];  // window 0 of the instance

  uint32_t acc[WPL];
#pragma unroll
  for (int e = 0; e < WPL; ++e) acc[e] = 0u;
  const bool mine = gl * WPL < nwords;  // this lane's words hold dense z of the row
  const int len = b - a;
  const int maxlen = wave_max(len);
  for (int c0 = 0; c0 < maxlen; c0 += LANES) {
    const int j = a + c0 + gl;
    const int code = (c0 + gl < len) ? c.rcode[j] : -1;
    // hot keys: one per group per step, four steps' loads in flight before the ORs
    const uint64_t hm = __ballot(code >= 0);
    uint64_t gm = LANES == 64 ? hm : (hm >> (grp * LANES)) & (~uint64_t(0) >> (64 - LANES));
    while (__ballot(gm != 0)) {
      uint32_t v[4][WPL];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool has = gm != 0;
        const int l = has ? __ffsll((unsigned long long)gm) - 1 : 0;
        const int k = __shfl(code, grp * LANES + l, 64);
#pragma unroll
        for (int e = 0; e < WPL; ++e) v[u][e] = 0u;
        if (has && mine) {
          const uint32_t* src = hrow + int64_t(k) * rw + gl * WPL;  // rows are whole windows: WPL words in bounds
          if constexpr (WPL == 8) {
            const uint4 q0 = reinterpret_cast<const uint4*>(src)[0], q1 = reinterpret_cast<const uint4*>(src)[1];
            const uint32_t w[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
            for (int e = 0; e < WPL; ++e) v[u][e] = w[e % 8];
          } else if constexpr (WPL == 4) {
            const uint4 q = *reinterpret_cast<const uint4*>(src);
            const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
            for (int e = 0; e < WPL; ++e) v[u][e] = w[e % 4];
          } else if constexpr (WPL == 2) {
            const uint2 q = *reinterpret_cast<const uint2*>(src);
            v[u][0] = q.x;
            v[u][WPL - 1] = q.y;
          } else {
            v[u][0] = src[0];
          }
        }
        gm &= gm - 1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int e = 0; e < WPL; ++e) acc[e] |= v[u][e];
    }
    // cold keys: the group scatters each key's window-0 entries (segment
    // bounds of four keys loaded together)
    const uint64_t cm = __ballot(code <= -2);
    uint64_t gc = LANES == 64 ? cm : (cm >> (grp * LANES)) & (~uint64_t(0) >> (64 - LANES));
    while (__ballot(gc != 0)) {
      int s0[4], s1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool has = gc != 0;
        const int l = has ? __ffsll((unsigned long long)gc) - 1 : 0;
        const int cd = __shfl(code, grp * LANES + l, 64);
        s0[u] = 0;
        s1[u] = 0;
        if (has) {
          const int yl = (-2 - cd) - yb;
          s0[u] = wp[yl];
          s1[u] = wp[yl + 1];
        }
        gc &= gc - 1;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        for (int t = s0[u] + gl; t < s1[u]; t += LANES) {
          const int dl = c.ccol[t];
          atomicOr(&buf[dl >> 5], 1u << (dl & 31));
        }
      }
    }
  }
  lds_fence();
  int pc = 0;
#pragma unroll
  for (int e = 0; e < WPL; ++e) pc += __popc(acc[e] | buf[gl * WPL + e]);
  if (!active) pc = 0;
#pragma unroll
  for (int o = LANES / 2; o > 0; o >>= 1) pc += __shfl_xor(pc, o, 64);
  if (active && gl == 0) {
    if (accumulate) atomicAdd(&cnt[x], pc);
    else cnt[x] = pc;
  }
}

// Algorithmic work of the count kernels (for roofline accounting):
// out[0] = sum_x hot(x) * words(x), out[1] = sum_x words(x),
// out[2] = sum_x cold dense entries of x, out[3] = sum_x w[x]
__global__ void k_work_stats(RowCtx c, int64_t x_lo, int64_t x_hi, const int64_t* __restrict__ w,
                             unsigned long long* __restrict__ out) {
  int64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int64_t b = x_lo + int64_t(blockIdx.x) * blockDim.x; b < x_hi; b += int64_t(gridDim.x) * blockDim.x) {
    const int64_t x = b + threadIdx.x;
    if (x < x_hi) {
      int inst = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.x_base, c.n_inst, int32_t(x));
      int zd = c.zd_base[inst + 1] - c.zd_base[inst];
      int64_t rw = int64_t((zd + 31) / 32);  // words of the dense range (window padding excluded)
      a1 += rw;
      a3 += w[x - x_lo];
    }
  }
  // per CSR entry (one thread each, so long rows do not serialise)
  const int64_t j_lo = c.rptr[x_lo], j_hi = c.rptr[x_hi];
  for (int64_t b = j_lo + int64_t(blockIdx.x) * blockDim.x; b < j_hi; b += int64_t(gridDim.x) * blockDim.x) {
    const int64_t j = b + threadIdx.x;
    if (j < j_hi) {
      const int code = c.rcode[j];
      if (code >= 0) {
        const int y = c.rcol[j];
        const int inst = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.y_base, c.n_inst, y);
        const int zd = c.zd_base[inst + 1] - c.zd_base[inst];
        a0 += int64_t((zd + 31) / 32);
      } else if (code <= -2) {
        a2 += c.cptr[-2 - code + 1] - c.cptr[-2 - code];
      }
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a3 = wave_sum(a3);
  if (lane_id() == 0) {
    atomicAdd(&out[0], (unsigned long long)a0);
    atomicAdd(&out[1], (unsigned long long)a1);
    atomicAdd(&out[2], (unsigned long long)a2);
    atomicAdd(&out[3], (unsigned long long)a3);
  }
}

// The same four sums over a list of rows (one thread per row), added to out.
__global__ void k_work_rows(RowCtx c, const int32_t* __restrict__ rows, int64_t n_rows,
                            const int64_t* __restrict__ w, unsigned long long* __restrict__ out) {
  int64_t a0 = 0, a1 = 0, a2 = 0, a3 = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n_rows; i += int64_t(gridDim.x) * blockDim.x) {
    const int32_t x = rows[i];
    const int inst = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.x_base, c.n_inst, x);
    const int zd = c.zd_base[inst + 1] - c.zd_base[inst];
    const int64_t words = int64_t((zd + 31) / 32);  // window padding excluded
    a1 += words;
    if (w) a3 += w[x];
    for (int j = c.rptr[x]; j < c.rptr[x + 1]; ++j) {
      const int code = c.rcode[j];
      if (code >= 0) a0 += words;
      else if (code <= -2) a2 += c.cptr[-2 - code + 1] - c.cptr[-2 - code];
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  a2 = wave_sum(a2);
  a3 = wave_sum(a3);
  if (lane_id() == 0) {
    atomicAdd(&out[0], (unsigned long long)a0);
    atomicAdd(&out[1], (unsigned long long)a1);
    atomicAdd(&out[2], (unsigned long long)a2);
    atomicAdd(&out[3], (unsigned long long)a3);
  }
}

}  // namespace

void work_rows(const RowCtx& c, const int32_t* rows, int64_t n_rows, const int64_t* w, int64_t* out4, hipStream_t s) {
  if (n_rows <= 0) return;
  int g = int(std::min<int64_t>((n_rows + NT - 1) / NT, 4096));
  hipLaunchKernelGGL(k_work_rows, dim3(g), dim3(NT), 0, s, c, rows, n_rows, w,
                     reinterpret_cast<unsigned long long*>(out4));
  JP_LAUNCH_CHECK();
}

// Windows per workgroup of the count kernel: as many as keep the hot-row
// slices of the windows in flight within about 512 KiB of an XCD's 4 MiB L2
// (each hot key holds DW_WORDS words per window).
int dense_window_group(int64_t max_hot, int nwin) {
  static const int env = [] {
    const char* e = std::getenv("JP_DENSE_WINDOW_GROUP");
    return e ? std::atoi(e) : 0;
  }();
  int64_t g = env > 0 ? env : (int64_t(1) << 19) / ((max_hot > 0 ? max_hot : 1) * DW_WORDS * 4);
  if (g < 1) g = 1;
  if (g > nwin) g = nwin > 0 ? nwin : 1;
  return int(g);
}

void work_stats(const RowCtx& c, int64_t x_lo, int64_t x_hi, const int64_t* w, int64_t* out4, hipStream_t s) {
  fill_i64(out4, 4, 0, s);
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  int g = int(std::min<int64_t>((n + NT - 1) / NT, 4096));
  hipLaunchKernelGGL(k_work_stats, dim3(g), dim3(NT), 0, s, c, x_lo, x_hi, w,
                     reinterpret_cast<unsigned long long*>(out4));
  JP_LAUNCH_CHECK();
}

// count of the rows of narrow instances (RowCtx::narrow), after the window
// kernel: all of them (rows == nullptr), or those in a list of n_rows rows
static void dense_narrow(const RowCtx& c, int64_t n_rows, const int32_t* rows, int accumulate, int32_t* cnt,
                         hipStream_t s) {
  if (c.narrow & 1) {
    const int64_t n = rows ? n_rows : c.nar_rows[0];
    hipLaunchKernelGGL((k_dense_narrow<8, 2>), dim3(int((n + 31) / 32)), dim3(256), 0, s, c, n, rows, accumulate, cnt);
    JP_LAUNCH_CHECK();
  }
  if (c.narrow & 2) {
    const int64_t n = rows ? n_rows : c.nar_rows[1];
    hipLaunchKernelGGL((k_dense_narrow<16, 4>), dim3(int((n + 15) / 16)), dim3(256), 0, s, c, n, rows, accumulate,
                       cnt);
    JP_LAUNCH_CHECK();
  }
  if (c.narrow & 4) {
    const int64_t n = rows ? n_rows : c.nar_rows[2];
    hipLaunchKernelGGL((k_dense_narrow<32, 8>), dim3(int((n + 7) / 8)), dim3(256), 0, s, c, n, rows, accumulate, cnt);
    JP_LAUNCH_CHECK();
  }
}

void dense_ec(const RowCtx& c, int64_t x_lo, int64_t x_hi, int32_t* cnt, const int64_t* off, int32_t* out,
              int64_t out_n, hipStream_t s) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  int g = int((n + RB - 1) / RB);
  if (out) {  // write mode emits each row's windows in order: one group
    hipLaunchKernelGGL(k_dense_bits<true>, dim3(g), dim3(NT), 0, s, c, x_lo, n, nullptr, nullptr, nullptr, 0, nullptr,
                       0, INT32_MAX, 0, cnt, off, out, out_n);
    JP_LAUNCH_CHECK();
  } else {
    const int nwin = int((c.max_zd_range + DW_BITS - 1) / DW_BITS);
    const int wg = c.wgroup > 0 ? std::max(1, std::min(c.wgroup, nwin)) : dense_window_group(c.max_hot, nwin);
    const int ng = (nwin + wg - 1) / wg;
    if (c.by_width) {
      // rows of instances without dense z keep 0; the window kernel counts the
      // rows of wide instances, the narrow kernels the others
      if (x_lo != 0 || x_hi != c.n_x) throw Error(JP_ESTATE, "rows listed by width are counted over the whole range");
      fill_i32(cnt, n, 0, s);
      const int64_t nw = c.nar_rows[N_WIDTH_CLASSES - 1];
      if (nw > 0) {
        hipLaunchKernelGGL(k_dense_bits<false>, dim3(int((nw + RB - 1) / RB), ng > 0 ? ng : 1), dim3(NT), 0, s, c,
                           int64_t(0), nw, nullptr, c.nar_base[N_WIDTH_CLASSES - 1], c.nar_x0[N_WIDTH_CLASSES - 1],
                           c.nar_m[N_WIDTH_CLASSES - 1], nullptr, 0, wg, 0, cnt,
                           off, out, int64_t(0));
        JP_LAUNCH_CHECK();
      }
      dense_narrow(c, 0, nullptr, 0, cnt, s);
    } else {
      if (ng > 1) fill_i32(cnt + x_lo, n, 0, s);
      hipLaunchKernelGGL(k_dense_bits<false>, dim3(g, ng > 0 ? ng : 1), dim3(NT), 0, s, c, x_lo, n, nullptr, nullptr,
                         nullptr, 0, nullptr, 0, wg, 0, cnt, off, out, int64_t(0));
      JP_LAUNCH_CHECK();
    }
  }
}

void dense_ec_rows(const RowCtx& c, const int32_t* rows, int64_t n_rows, const int32_t* base_cnt, int32_t* cnt,
                   hipStream_t s) {
  if (n_rows <= 0) return;
  const int g = int((n_rows + RB - 1) / RB);
  const int nwin = int((c.max_zd_range + DW_BITS - 1) / DW_BITS);
  const int wg = c.wgroup > 0 ? std::max(1, std::min(c.wgroup, nwin)) : dense_window_group(c.max_hot, nwin);
  const int ng = (nwin + wg - 1) / wg;
  // with a base count (rows outside a pivot) every row stays in the window kernel
  const int skip = (c.narrow && !base_cnt) ? 1 : 0;
  hipLaunchKernelGGL(k_dense_bits<false>, dim3(g, ng > 0 ? ng : 1), dim3(NT), 0, s, c, int64_t(0), n_rows, rows,
                     nullptr, nullptr, 0, base_cnt, 1, wg, skip, cnt, nullptr, nullptr, int64_t(0));
  JP_LAUNCH_CHECK();
  if (skip) dense_narrow(c, n_rows, rows, 1, cnt, s);
}

}  // namespace jp
