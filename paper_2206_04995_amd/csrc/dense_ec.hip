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

// Rows are slots [0, n_rows): slot i is row rows[i] (a list, count mode) or
// x_lo + i.  In count mode the row's count starts at base_cnt[instance] (the
// pivot row's size when the rows are evaluated outside the pivot's z) and is
// stored, or added when the grid has several window groups or `accumulate`.
template <bool WRITE>
__global__ void __launch_bounds__(NT, 8) k_dense_bits(RowCtx c, int64_t x_lo, int64_t n_rows,
                                                   const int32_t* __restrict__ rows,
                                                   const int32_t* __restrict__ base_cnt, int accumulate, int wgroup,
                                                   int32_t* __restrict__ cnt, const int64_t* __restrict__ off,
                                                   int32_t* __restrict__ out, int64_t out_n) {
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

  // instance of the block's first row: its hottest keys are staged in LDS
  const int64_t xb0 = rows ? int64_t(rows[rb0]) : x_lo + rb0;
  const int inst0 = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.x_base, c.n_inst, int32_t(xb0));
  const int zd0 = c.zd_base[inst0 + 1] - c.zd_base[inst0];
  const int nwin0 = (zd0 + DW_BITS - 1) / DW_BITS;
  const int k0 = c.Ehot[c.y_base[inst0 + 1]] - c.Ehot[c.y_base[inst0]];
  const int t_eff = k0 < T_STAGE ? k0 : T_STAGE;
  const uint32_t* hb0 = c.hb + c.hb_off[inst0];
  const int64_t rw0 = c.row_words[inst0];

  // lane r < nrows describes row r0 + r
  int my_inst = 0, my_nwin = 0, my_a = 0, my_b = 0;
  int64_t my_x = 0;
  int64_t my_acc = 0;  // count (count mode) or write position (write mode)
  if (lane < nrows) {
    const int64_t x = rows ? int64_t(rows[r0 + lane]) : x_lo + r0 + lane;
    my_x = x;
    my_inst = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.x_base, c.n_inst, int32_t(x));
    const int zd = c.zd_base[my_inst + 1] - c.zd_base[my_inst];
    my_nwin = (zd + DW_BITS - 1) / DW_BITS;
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
      for (int i = threadIdx.x; i < t_eff * QW; i += NT) {
        const int k = i / QW, q = i - k * QW;
        stage[k][q] = reinterpret_cast<const uint4*>(hb0 + int64_t(k) * rw0 + int64_t(w) * DW_WORDS)[q];
      }
    }
    __syncthreads();

#pragma unroll
    for (int r = 0; r < RPW; ++r) {
      if (r >= nrows) break;
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

      // bounds of this window's cold segments: issued first, used after the hot ORs
      const int cd = code[r];
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
      hot_or<Q>(acc, cd, staged, t_eff, stage, hbase, rw);
      for (int c0 = a + 64; c0 < b; c0 += 64) {  // rows with more than 64 join keys
        const int j = c0 + lane;
        const int cx = j < b ? c.rcode[j] : -1;
        any_cold |= ballot(cx <= -2) != 0;
        hot_or<Q>(acc, cx, staged, t_eff, stage, hbase, rw);
      }
      if (any_cold) {
#pragma unroll
        for (int q = 0; q < Q; ++q) rowbuf4[q * 64 + lane] = acc[q];
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
        for (int q = 0; q < Q; ++q) acc[q] = rowbuf4[q * 64 + lane];
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
      int64_t rw = zd > 0 ? int64_t((zd + DW_BITS - 1) / DW_BITS) * DW_WORDS : 0;
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
        a0 += int64_t((zd + DW_BITS - 1) / DW_BITS) * DW_WORDS;
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
    const int64_t words = zd > 0 ? int64_t((zd + DW_BITS - 1) / DW_BITS) * DW_WORDS : 0;
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

void dense_ec(const RowCtx& c, int64_t x_lo, int64_t x_hi, int32_t* cnt, const int64_t* off, int32_t* out,
              int64_t out_n, hipStream_t s) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  int g = int((n + RB - 1) / RB);
  if (out) {  // write mode emits each row's windows in order: one group
    hipLaunchKernelGGL(k_dense_bits<true>, dim3(g), dim3(NT), 0, s, c, x_lo, n, nullptr, nullptr, 0, INT32_MAX, cnt,
                       off, out, out_n);
  } else {
    const int nwin = int((c.max_zd_range + DW_BITS - 1) / DW_BITS);
    const int wg = c.wgroup > 0 ? std::max(1, std::min(c.wgroup, nwin)) : dense_window_group(c.max_hot, nwin);
    const int ng = (nwin + wg - 1) / wg;
    if (ng > 1) fill_i32(cnt + x_lo, n, 0, s);
    hipLaunchKernelGGL(k_dense_bits<false>, dim3(g, ng > 0 ? ng : 1), dim3(NT), 0, s, c, x_lo, n, nullptr, nullptr, 0,
                       wg, cnt, off, out, int64_t(0));
  }
  JP_LAUNCH_CHECK();
}

void dense_ec_rows(const RowCtx& c, const int32_t* rows, int64_t n_rows, const int32_t* base_cnt, int32_t* cnt,
                   hipStream_t s) {
  if (n_rows <= 0) return;
  const int g = int((n_rows + RB - 1) / RB);
  const int nwin = int((c.max_zd_range + DW_BITS - 1) / DW_BITS);
  const int wg = c.wgroup > 0 ? std::max(1, std::min(c.wgroup, nwin)) : dense_window_group(c.max_hot, nwin);
  const int ng = (nwin + wg - 1) / wg;
  hipLaunchKernelGGL(k_dense_bits<false>, dim3(g, ng > 0 ? ng : 1), dim3(NT), 0, s, c, int64_t(0), n_rows, rows,
                     base_cnt, 1, wg, cnt, nullptr, nullptr, int64_t(0));
  JP_LAUNCH_CHECK();
}

}  // namespace jp
