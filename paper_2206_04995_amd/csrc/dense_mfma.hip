// DenseEC on the INT8 matrix cores (paper Sec. 2.5): for a dense panel the
// dense part is the 0/1 product C = A * B over the instance's dense join keys,
// A[x][k] = [(x, y_k) in R], B[k][z] = [(z, y_k) in S_dense], and a pair (x, z)
// is in the result iff C[x][z] > 0.  Counts never exceed the number of keys
// (< 2^31), so int32 accumulation and the test > 0 are exact.
//
// A is stored x-major and B transposed (z-major), both with the key index
// contiguous, so one 16-byte load gives a lane its 16 k-values of an MFMA
// operand.  A workgroup of WR x WC waves computes a tile of C, each wave a
// (16 TI) x (16 TJ) block of v_mfma_i32_16x16x64_i8.  Every step stages KT
// keys of both panels in LDS, double buffered: the next step's loads are in
// flight while the current step multiplies.  LDS rows carry one 16-byte chunk
// of padding so the 16-byte operand reads of 16 consecutive rows fall in
// distinct banks.  Lane l of a 16x16x64 operand holds row (or column) l % 16
// and keys 16 * (l / 16) .. + 15; its accumulator element r is
// C[4 * (l / 16) + r][l % 16].  The epilogue counts C > 0 per row with ballots
// and adds one partial count per row and tile.
//
// Early check (the early stop of the paper's DenseEC, Sec. 2.5): the products
// are 0/1, so a sum only grows; once every entry of a workgroup's tile is > 0
// the remaining keys cannot change any decision.  Every CHECK_EVERY staged
// steps each wave votes whether all its entries (rows and columns past the
// panel count as decided) are > 0, and the workgroup stops when all vote yes.
// The staged steps a workgroup ran are added to *steps, for the issued work.
#include "common.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

// wave tile (16 * TI) x (16 * TJ), WR x WC waves per workgroup
constexpr int TI = 4, TJ = 8, WR = 4, WC = 2;
constexpr int MT = WR * 16 * TI;  // x rows per workgroup tile
constexpr int ZT = WC * 16 * TJ;  // dense z per workgroup tile
constexpr int KS = 2;             // 64-key MFMA steps per staged step
constexpr int KT = 64 * KS;       // keys per staged step
constexpr int CPR = KT / 16;      // 16-byte chunks per panel row and step
constexpr int BT = 64 * WR * WC;  // threads per workgroup
constexpr int RP = CPR + 1;       // 16-byte chunks per LDS row (one of padding)
constexpr int SA = MT * CPR / BT;  // 16-byte staging loads per thread and step, panel A
constexpr int SB = ZT * CPR / BT;  // the same for panel B
constexpr int CHECK_EVERY = 4;     // staged steps between early checks
static_assert(SA >= 1 && SB >= 1 && MT * CPR % BT == 0 && ZT * CPR % BT == 0, "staging split");

template <int TI, int TJ>
__global__ void __launch_bounds__(BT, 1) k_dense_mfma(const int8_t* __restrict__ A, const int8_t* __restrict__ Bt,
                                                      int64_t k_pad, int64_t nx, int64_t nz, int32_t* __restrict__ cnt,
                                                      unsigned long long* __restrict__ steps) {
  constexpr int MT = WR * 16 * TI;   // x rows of this tile
  constexpr int ZT = WC * 16 * TJ;   // dense z of this tile
  constexpr int SA = MT * CPR / BT;  // 16-byte staging loads per thread and step, panel A
  constexpr int SB = ZT * CPR / BT;  // the same for panel B
  static_assert(SA >= 1 && SB >= 1 && MT * CPR % BT == 0 && ZT * CPR % BT == 0, "staging split");
  __shared__ v4i As[2][MT * RP];
  __shared__ v4i Bs[2][ZT * RP];
  __shared__ int s_full[2][WR * WC];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid / WC, wc = wid % WC;
  const int64_t x0 = int64_t(blockIdx.y) * MT, z0 = int64_t(blockIdx.x) * ZT;
  v4i acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = v4i{0, 0, 0, 0};

  // staging chunk c of a panel: row c / 4, 16-byte column c % 4
  v4i pa[SA], pb[SB];
#pragma unroll
  for (int s = 0; s < SA; ++s) {
    const int c = tid + s * BT;
    pa[s] = *reinterpret_cast<const v4i*>(A + (x0 + (c / CPR)) * k_pad + (c % CPR) * 16);
    As[0][(c / CPR) * RP + (c % CPR)] = pa[s];
  }
#pragma unroll
  for (int s = 0; s < SB; ++s) {
    const int c = tid + s * BT;
    pb[s] = *reinterpret_cast<const v4i*>(Bt + (z0 + (c / CPR)) * k_pad + (c % CPR) * 16);
    Bs[0][(c / CPR) * RP + (c % CPR)] = pb[s];
  }
  __syncthreads();
  const int nk = int(k_pad / KT);
  const int g = lane >> 4;
  int ran = nk;
  for (int ks = 0; ks < nk; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < nk) {
      const int64_t kk = int64_t(ks + 1) * KT;
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int c = tid + s * BT;
        pa[s] = *reinterpret_cast<const v4i*>(A + (x0 + (c / CPR)) * k_pad + kk + (c % CPR) * 16);
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int c = tid + s * BT;
        pb[s] = *reinterpret_cast<const v4i*>(Bt + (z0 + (c / CPR)) * k_pad + kk + (c % CPR) * 16);
      }
    }
#pragma unroll
    for (int kq = 0; kq < KS; ++kq) {
      v4i a[TI], b[TJ];
#pragma unroll
      for (int t = 0; t < TI; ++t) a[t] = As[cur][(wr * 16 * TI + t * 16 + (lane & 15)) * RP + 4 * kq + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < TJ; ++t) b[t] = Bs[cur][(wc * 16 * TJ + t * 16 + (lane & 15)) * RP + 4 * kq + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (ks + 1 < nk) {
#pragma unroll
      for (int s = 0; s < SA; ++s) {
        const int c = tid + s * BT;
        As[cur ^ 1][(c / CPR) * RP + (c % CPR)] = pa[s];
      }
#pragma unroll
      for (int s = 0; s < SB; ++s) {
        const int c = tid + s * BT;
        Bs[cur ^ 1][(c / CPR) * RP + (c % CPR)] = pb[s];
      }
    }
    const bool check = (ks + 1) % CHECK_EVERY == 0 && ks + 1 < nk;
    const int par = (ks / CHECK_EVERY) & 1;
    if (check) {
      bool full = true;
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t x = x0 + wr * 16 * TI + i * 16 + 4 * g + r;
            const int64_t z = z0 + wc * 16 * TJ + j * 16 + (lane & 15);
            full = full && (acc[i][j][r] > 0 || x >= nx || z >= nz);
          }
      const bool wave_full = ballot(!full) == 0;
      if (lane == 0) s_full[par][wid] = wave_full ? 1 : 0;
    }
    __syncthreads();
    if (check) {
      bool all = true;
#pragma unroll
      for (int w = 0; w < WR * WC; ++w) all = all && s_full[par][w] != 0;
      if (all) {
        ran = ks + 1;
        break;
      }
    }
  }
  if (tid == 0) atomicAdd(steps, (unsigned long long)ran);

#pragma unroll
  for (int i = 0; i < TI; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int c = 0;
#pragma unroll
      for (int j = 0; j < TJ; ++j) {
        const uint64_t m = ballot(acc[i][j][r] > 0);
        c += __popcll((m >> (16 * g)) & 0xFFFFull);
      }
      const int64_t x = x0 + wr * 16 * TI + i * 16 + 4 * g + r;
      if ((lane & 15) == 0 && x < nx && c) atomicAdd(&cnt[x], c);
    }
  }
}

// key index of every join key with a dense S entry (-1 otherwise)
// key index of every join key with a dense S entry and an R row (-1 otherwise)
__global__ void k_panel_keys(const int32_t* __restrict__ sptr, const int32_t* __restrict__ spptr,
                             const int32_t* __restrict__ dR, const int32_t* __restrict__ E, int64_t n_y,
                             int32_t* __restrict__ kmap) {
  for (int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; y < n_y; y += int64_t(gridDim.x) * blockDim.x) {
    const int dd = (sptr[y + 1] - sptr[y]) - (spptr[y + 1] - spptr[y]);
    kmap[y] = (dd > 0 && dR[y] > 0) ? E[y] : -1;
  }
}

__global__ void k_panel_key_flags(const int32_t* __restrict__ sptr, const int32_t* __restrict__ spptr,
                                  const int32_t* __restrict__ dR, int64_t n_y, int32_t* __restrict__ flag) {
  for (int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; y < n_y; y += int64_t(gridDim.x) * blockDim.x)
    flag[y] = (((sptr[y + 1] - sptr[y]) - (spptr[y + 1] - spptr[y])) > 0 && dR[y] > 0) ? 1 : 0;
}

// A[x][kmap[y]] = 1 for every R entry (one wavefront per row)
__global__ void k_panel_a(const int32_t* __restrict__ rptr, const int32_t* __restrict__ rcol, int64_t n_x,
                          const int32_t* __restrict__ kmap, int64_t k_pad, int8_t* __restrict__ A) {
  const int lane = lane_id();
  const int64_t waves = int64_t(gridDim.x) * (blockDim.x >> 6);
  for (int64_t x = int64_t(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6); x < n_x; x += waves) {
    for (int j = rptr[x] + lane; j < rptr[x + 1]; j += 64) {
      const int k = kmap[rcol[j]];
      if (k >= 0) A[x * k_pad + k] = 1;
    }
  }
}

// Bt[dense z][kmap[y]] = 1 for every dense S entry (one thread per entry)
__global__ void k_panel_bt(const int32_t* __restrict__ Ey, const int32_t* __restrict__ scol, int64_t n,
                           const int32_t* __restrict__ zflag, const int32_t* __restrict__ Edz,
                           const int32_t* __restrict__ kmap, int64_t k_pad, int8_t* __restrict__ Bt) {
  for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < n; p += int64_t(gridDim.x) * blockDim.x) {
    const int32_t z = scol[p];
    if (!zflag[z]) continue;
    const int k = kmap[Ey[p + 1] - 1];
    if (k >= 0) Bt[int64_t(Edz[z]) * k_pad + k] = 1;
  }
}

inline int grid256(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16))); }

}  // namespace

int64_t panel_key_count(const int32_t* sptr, const int32_t* spptr, const int32_t* dR, int64_t n_y, int32_t* kmap,
                        Arena& T, hipStream_t s) {
  if (n_y <= 0) return 0;
  int32_t* flag = T.alloc<int32_t>(n_y, s);
  hipLaunchKernelGGL(k_panel_key_flags, dim3(grid256(n_y)), dim3(256), 0, s, sptr, spptr, dR, n_y, flag);
  JP_LAUNCH_CHECK();
  int32_t* E = T.alloc<int32_t>(n_y + 1, s);
  scan_excl_i32(flag, E, n_y, s, T);
  hipLaunchKernelGGL(k_panel_keys, dim3(grid256(n_y)), dim3(256), 0, s, sptr, spptr, dR, E, n_y, kmap);
  JP_LAUNCH_CHECK();
  int32_t k = 0;
  JP_HIP(hipMemcpyAsync(&k, E + n_y, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));
  return k;
}

void build_panels(const int32_t* rptr, const int32_t* rcol, int64_t n_x, const int32_t* Ey, const int32_t* scol,
                  int64_t n_s, const int32_t* zflag, const int32_t* Edz, const int32_t* kmap, int64_t k_pad,
                  int64_t nx_pad, int64_t nz_pad, int8_t* A, int8_t* Bt, hipStream_t s) {
  fill_u32(reinterpret_cast<uint32_t*>(A), nx_pad * k_pad / 4, 0u, s);
  fill_u32(reinterpret_cast<uint32_t*>(Bt), nz_pad * k_pad / 4, 0u, s);
  if (n_x > 0) {
    hipLaunchKernelGGL(k_panel_a, dim3(grid256(n_x * 64)), dim3(256), 0, s, rptr, rcol, n_x, kmap, k_pad, A);
    JP_LAUNCH_CHECK();
  }
  if (n_s > 0) {
    hipLaunchKernelGGL(k_panel_bt, dim3(grid256(n_s)), dim3(256), 0, s, Ey, scol, n_s, zflag, Edz, kmap, k_pad, Bt);
    JP_LAUNCH_CHECK();
  }
}

int64_t mfma_pad_rows(int64_t n) { return (n + MT - 1) / MT * MT; }
int64_t mfma_pad_keys(int64_t n) { return (n + KT - 1) / KT * KT; }
int64_t mfma_pad_cols(int64_t n) { return (n + ZT - 1) / ZT * ZT; }

// tile 0: 256 x 256 (4 x 8 MFMA blocks per wave), 1: 128 x 256 (2 x 8), 2: 256 x 128 (4 x 4)
void dense_mfma_count(const int8_t* A, const int8_t* Bt, int64_t k_pad, int64_t nx, int64_t nx_pad, int64_t nz,
                      int64_t nz_pad, int32_t* cnt, int64_t* steps, int tile, hipStream_t s) {
  fill_i32(cnt, nx, 0, s);
  fill_i64(steps, 1, 0, s);
  if (nx <= 0 || nz_pad <= 0 || k_pad <= 0) return;
  const int mt = tile == 1 ? MT / 2 : MT, zt = tile == 2 ? ZT / 2 : ZT;
  dim3 grid(unsigned(nz_pad / zt), unsigned(nx_pad / mt));  // padded by mfma_pad_rows / mfma_pad_cols
  auto* st = reinterpret_cast<unsigned long long*>(steps);
  if (tile == 1)
    hipLaunchKernelGGL((k_dense_mfma<2, 8>), grid, dim3(BT), 0, s, A, Bt, k_pad, nx, nz, cnt, st);
  else if (tile == 2)
    hipLaunchKernelGGL((k_dense_mfma<4, 4>), grid, dim3(BT), 0, s, A, Bt, k_pad, nx, nz, cnt, st);
  else
    hipLaunchKernelGGL((k_dense_mfma<4, 8>), grid, dim3(BT), 0, s, A, Bt, k_pad, nx, nz, cnt, st);
  JP_LAUNCH_CHECK();
}

int64_t mfma_step_ops(int tile) {
  const int64_t mt = tile == 1 ? MT / 2 : MT, zt = tile == 2 ? ZT / 2 : ZT;
  return 2 * mt * zt * KT;
}

}  // namespace jp
