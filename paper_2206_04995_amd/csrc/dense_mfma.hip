// DenseEC on the INT8 matrix cores (paper Sec. 2.5): for a dense panel the
// dense part is the 0/1 product C = A * B over the instance's dense join keys,
// A[x][k] = [(x, y_k) in R], B[k][z] = [(z, y_k) in S_dense], and a pair (x, z)
// is in the result iff C[x][z] > 0.  Counts never exceed the number of keys
// (< 2^31), so int32 accumulation and the test > 0 are exact.
//
// A is stored x-major and B transposed (z-major), both with the key index
// contiguous, so one 16-byte load gives a lane its 16 k-values of an MFMA
// operand.  A workgroup computes a 128 x 128 tile of C with four waves of
// 64 x 64 (4 x 4 blocks of v_mfma_i32_16x16x64_i8), staging 64 keys of both
// panels per step in LDS.  Lane l of a 16x16x64 operand holds row (or column)
// l % 16 and keys 16 * (l / 16) .. + 15; its accumulator element r is
// C[4 * (l / 16) + r][l % 16].  The epilogue counts C > 0 per row with
// ballots and adds one partial count per row and tile.
#include "common.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int MT = 128;  // x rows per workgroup tile
constexpr int ZT = 128;  // dense z per workgroup tile
constexpr int KT = 64;   // keys per step
constexpr int BT = 256;  // 4 waves: 2 x 2 quadrants of 64 x 64

__global__ void __launch_bounds__(BT) k_dense_mfma(const int8_t* __restrict__ A, const int8_t* __restrict__ Bt,
                                                   int64_t k_pad, int64_t nx, int32_t* __restrict__ cnt) {
  __shared__ v4i As[MT][KT / 16];
  __shared__ v4i Bs[ZT][KT / 16];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = wid >> 1, wc = wid & 1;
  const int64_t x0 = int64_t(blockIdx.y) * MT, z0 = int64_t(blockIdx.x) * ZT;
  v4i acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4i{0, 0, 0, 0};

  for (int64_t k0 = 0; k0 < k_pad; k0 += KT) {
#pragma unroll
    for (int c = tid; c < MT * (KT / 16); c += BT) {
      const int r = c >> 2, q = c & 3;
      As[r][q] = *reinterpret_cast<const v4i*>(A + (x0 + r) * k_pad + k0 + q * 16);
      Bs[r][q] = *reinterpret_cast<const v4i*>(Bt + (z0 + r) * k_pad + k0 + q * 16);
    }
    __syncthreads();
    v4i a[4], b[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a[t] = As[wr * 64 + t * 16 + (lane & 15)][lane >> 4];
      b[t] = Bs[wc * 64 + t * 16 + (lane & 15)][lane >> 4];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  const int g = lane >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int c = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint64_t m = ballot(acc[i][j][r] > 0);
        c += __popcll((m >> (16 * g)) & 0xFFFFull);
      }
      const int64_t x = x0 + wr * 64 + i * 16 + 4 * g + r;
      if ((lane & 15) == 0 && x < nx && c) atomicAdd(&cnt[x], c);
    }
  }
}

// key index of every join key with a dense S entry (-1 otherwise)
__global__ void k_panel_keys(const int32_t* __restrict__ sptr, const int32_t* __restrict__ spptr,
                             const int32_t* __restrict__ E, int64_t n_y, int32_t* __restrict__ kmap) {
  for (int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; y < n_y; y += int64_t(gridDim.x) * blockDim.x) {
    const int dd = (sptr[y + 1] - sptr[y]) - (spptr[y + 1] - spptr[y]);
    kmap[y] = dd > 0 ? E[y] : -1;
  }
}

__global__ void k_panel_key_flags(const int32_t* __restrict__ sptr, const int32_t* __restrict__ spptr, int64_t n_y,
                                  int32_t* __restrict__ flag) {
  for (int64_t y = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; y < n_y; y += int64_t(gridDim.x) * blockDim.x)
    flag[y] = ((sptr[y + 1] - sptr[y]) - (spptr[y + 1] - spptr[y])) > 0 ? 1 : 0;
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

int64_t panel_key_count(const int32_t* sptr, const int32_t* spptr, int64_t n_y, int32_t* kmap, Arena& T,
                        hipStream_t s) {
  if (n_y <= 0) return 0;
  int32_t* flag = T.alloc<int32_t>(n_y, s);
  hipLaunchKernelGGL(k_panel_key_flags, dim3(grid256(n_y)), dim3(256), 0, s, sptr, spptr, n_y, flag);
  JP_LAUNCH_CHECK();
  int32_t* E = T.alloc<int32_t>(n_y + 1, s);
  scan_excl_i32(flag, E, n_y, s, T);
  hipLaunchKernelGGL(k_panel_keys, dim3(grid256(n_y)), dim3(256), 0, s, sptr, spptr, E, n_y, kmap);
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

void dense_mfma_count(const int8_t* A, const int8_t* Bt, int64_t k_pad, int64_t nx, int64_t nx_pad, int64_t nz_pad,
                      int32_t* cnt, hipStream_t s) {
  fill_i32(cnt, nx, 0, s);
  if (nx <= 0 || nz_pad <= 0 || k_pad <= 0) return;
  dim3 grid(unsigned(nz_pad / ZT), unsigned(nx_pad / MT));
  hipLaunchKernelGGL(k_dense_mfma, grid, dim3(BT), 0, s, A, Bt, k_pad, nx, cnt);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
