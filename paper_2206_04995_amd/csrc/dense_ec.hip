// DenseEC (paper Sec. 2.5, Alg. 3) for the dense z's of the partition:
// C[x, z] = OR over y of R[x, y] AND S[y, z].
//
// The paper tests one (x, z) pair at a time, either by a SIMD AND of the two
// |Y|-bit bitmaps or by probing Bitmap_z at each y of x, stopping at the
// first hit.  Here one wavefront builds a whole window of the x row at once:
// the row's "hot" join keys (y with many dense S entries) are kept as bit rows
// over the dense z index and are ORed word by word (32 z per lane-op), and the
// remaining "cold" keys are scattered from their z-sorted CSR rows into an
// LDS copy of the window.  The window is then popcounted (count mode) or
// written out in z order (write mode).
//
// Rows run in blocks of 16 per wavefront; all rows of a block walk the
// windows in the same order so the hot rows' window slices are reused from
// the caches, and each (row, cold y) keeps a cursor into its cold row across
// windows, so a cold entry is read once.
#include "common.h"
#include "stages.h"

namespace jp {
namespace {

constexpr int NT = 256;
constexpr int WAVES = NT / 64;
constexpr int RPW = 16;                   // rows per wavefront
constexpr int WPL = DW_WORDS / 64;        // words of a window per lane (16)
constexpr int Q = WPL / 4;                // uint4 per lane (4)

__device__ __forceinline__ void lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int popc4(uint4 v) { return __popc(v.x) + __popc(v.y) + __popc(v.z) + __popc(v.w); }

template <bool WRITE>
__global__ void __launch_bounds__(NT) k_dense_bits(RowCtx c, int64_t x_lo, int64_t x_hi, int32_t* __restrict__ cnt,
                                                   const int64_t* __restrict__ off, int32_t* __restrict__ out) {
  __shared__ uint4 rowbuf_all[WAVES][DW_WORDS / 4];
  __shared__ int32_t curs_all[WAVES][RPW][64];
  const int lane = lane_id();
  const int wid = threadIdx.x >> 6;
  uint32_t* rowbuf = reinterpret_cast<uint32_t*>(rowbuf_all[wid]);
  uint4* rowbuf4 = rowbuf_all[wid];
  int32_t(*curs)[64] = curs_all[wid];

  const int64_t r0 = x_lo + (int64_t(blockIdx.x) * WAVES + wid) * RPW;
  if (r0 >= x_hi) return;
  const int nrows = int((x_hi - r0) < RPW ? (x_hi - r0) : RPW);
  const int64_t base_off = WRITE ? off[x_lo] : 0;

  // lane r < nrows describes row r0 + r
  int my_inst = 0, my_nwin = 0;
  int64_t my_acc = 0;  // count (count mode) or write position (write mode)
  if (lane < nrows) {
    int64_t x = r0 + lane;
    my_inst = c.n_inst == 1 ? 0 : find_inst<int32_t>(c.x_base, c.n_inst, int32_t(x));
    int zd = c.zd_base[my_inst + 1] - c.zd_base[my_inst];
    my_nwin = (zd + DW_BITS - 1) / DW_BITS;
    if (WRITE) my_acc = off[x] - base_off;
  }
  const int maxwin = wave_max(my_nwin);
  if (maxwin == 0) {
    if (!WRITE && lane < nrows) cnt[r0 + lane] = 0;
    return;
  }

  // cursors of the first 64 join keys of each row into their cold rows
  for (int r = 0; r < nrows; ++r) {
    const int64_t x = r0 + r;
    const int a = c.rptr[x], b = c.rptr[x + 1];
    int cur = -1;
    if (a + lane < b) {
      int y = c.rcol[a + lane];
      if (c.hotrow[y] < 0 && c.cptr[y + 1] > c.cptr[y]) cur = c.cptr[y];
    }
    curs[r][lane] = cur;
  }
  lds_fence();

  for (int w = 0; w < maxwin; ++w) {
    const int32_t wstart = w * DW_BITS;
    const int32_t wend = wstart + DW_BITS;
    for (int r = 0; r < nrows; ++r) {
      const int nwin_r = __shfl(my_nwin, r, 64);
      if (w >= nwin_r) continue;
      const int inst = __shfl(my_inst, r, 64);
      const int64_t x = r0 + r;
      const int a = c.rptr[x], b = c.rptr[x + 1];
      const uint32_t* hbase = c.hb + c.hb_off[inst] + int64_t(w) * DW_WORDS;
      const int64_t rw = c.row_words[inst];

      uint4 acc[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) acc[q] = make_uint4(0, 0, 0, 0);
      bool any_cold = false;
      for (int c0 = a; c0 < b; c0 += 64) {
        const int j = c0 + lane;
        int y = -1, hr = -1;
        bool cold = false;
        if (j < b) {
          y = c.rcol[j];
          hr = c.hotrow[y];
          cold = hr < 0 && c.cptr[y + 1] > c.cptr[y];
        }
        uint64_t hm = ballot(hr >= 0);
        any_cold |= ballot(cold) != 0;
        while (hm) {
          const int l = __ffsll((unsigned long long)hm) - 1;
          hm &= hm - 1;
          const int k = __shfl(hr, l, 64);
          const uint4* src = reinterpret_cast<const uint4*>(hbase + int64_t(k) * rw);
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            uint4 v = src[q * 64 + lane];
            acc[q].x |= v.x;
            acc[q].y |= v.y;
            acc[q].z |= v.z;
            acc[q].w |= v.w;
          }
        }
      }
      if (any_cold) {
#pragma unroll
        for (int q = 0; q < Q; ++q) rowbuf4[q * 64 + lane] = acc[q];
        lds_fence();
        int ci = 0;
        for (int c0 = a; c0 < b; c0 += 64, ++ci) {
          const int j = c0 + lane;
          if (j < b) {
            const int y = c.rcol[j];
            if (c.hotrow[y] < 0) {
              const int c1 = c.cptr[y + 1];
              int cur;
              if (ci == 0) {
                cur = curs[r][lane];
              } else {
                const int cs = c.cptr[y];
                cur = cs < c1 ? int(lower_bound_dev<int32_t>(c.ccol, cs, c1, wstart)) : -1;
              }
              if (cur >= 0) {
                while (cur < c1) {
                  const int32_t d = c.ccol[cur];
                  if (d >= wend) break;
                  const int dl = d - wstart;
                  atomicOr(&rowbuf[dl >> 5], 1u << (dl & 31));
                  ++cur;
                }
                if (ci == 0) curs[r][lane] = cur < c1 ? cur : -1;
              }
            }
          }
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
        const int tot = wave_sum(pc);
        if (lane == r) my_acc += tot;
      } else {
        int64_t pos0 = __shfl(my_acc, r, 64);
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
              out[pos++] = c.dz2z[dzb + wbase + bit];
            }
          }
          qbase += tq;
        }
        if (lane == r) my_acc += qbase;
      }
    }
  }
  if (!WRITE && lane < nrows) cnt[r0 + lane] = int32_t(my_acc);
}

}  // namespace

void dense_ec(const RowCtx& c, int64_t x_lo, int64_t x_hi, int32_t* cnt, const int64_t* off, int32_t* out,
              hipStream_t s) {
  int64_t n = x_hi - x_lo;
  if (n <= 0) return;
  int64_t rows_per_block = int64_t(WAVES) * RPW;
  int g = int((n + rows_per_block - 1) / rows_per_block);
  if (out)
    hipLaunchKernelGGL(k_dense_bits<true>, dim3(g), dim3(NT), 0, s, c, x_lo, x_hi, cnt, off, out);
  else
    hipLaunchKernelGGL(k_dense_bits<false>, dim3(g), dim3(NT), 0, s, c, x_lo, x_hi, cnt, off, out);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
