// Union of the two parts and output (paper Alg. 1, last step): the dense and
// sparse results are disjoint by construction of the partition, so per-row
// counts add and the sorted row lists merge without deduplication.
#include "common.h"
#include "prim.h"
#include "stages.h"

namespace jp {
namespace {

constexpr int NT = 256;

__global__ void k_add_counts(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n,
                             int32_t* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = a[i] + b[i];
}

// per-instance totals straight from the per-row counts (no offsets):
// tot[3i] += dense + sparse, tot[3i + 1] += dense, tot[3i + 2] += sparse over
// the rows of instance i (tot zeroed before).  A thread sums its rows of one
// instance at a time; at the end a wave whose lanes all hold the same
// instance adds once.
__device__ __forceinline__ void add_tot(int64_t* tot, int inst, int64_t de, int64_t sp) {
  atomicAdd(reinterpret_cast<unsigned long long*>(&tot[3 * inst + 0]), (unsigned long long)(de + sp));
  atomicAdd(reinterpret_cast<unsigned long long*>(&tot[3 * inst + 1]), (unsigned long long)de);
  atomicAdd(reinterpret_cast<unsigned long long*>(&tot[3 * inst + 2]), (unsigned long long)sp);
}

__global__ void k_inst_sums(const int32_t* __restrict__ cnt_sp, const int32_t* __restrict__ cnt_de,
                            const int32_t* __restrict__ x_base, int n_inst, int64_t n_x, int64_t* __restrict__ tot) {
  SegCursor<int32_t> cur(x_base, n_inst);
  cur.seed(int32_t(chunk_first() < n_x ? chunk_first() : 0));
  int acc = -1;
  int64_t de = 0, sp = 0;
  CHUNK_LOOP(x, n_x, JP_CHUNK) {
    const int inst = cur(int32_t(x));
    if (inst != acc) {
      if (acc >= 0) add_tot(tot, acc, de, sp);
      acc = inst;
      de = 0;
      sp = 0;
    }
    de += cnt_de[x];
    sp += cnt_sp[x];
  }
  const int i0 = __builtin_amdgcn_readfirstlane(acc);
  if (ballot(acc != i0) == 0) {
    de = wave_sum(de);
    sp = wave_sum(sp);
    if (lane_id() == 0 && acc >= 0) add_tot(tot, acc, de, sp);
  } else if (acc >= 0) {
    add_tot(tot, acc, de, sp);
  }
}

// out2[0] = row holding pair g0, out2[1] = first row starting at or after g1
__global__ void k_find_rows(const int64_t* __restrict__ off, int64_t xb, int64_t xe, int64_t g0, int64_t g1,
                            int64_t* __restrict__ out2) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // largest x in [xb, xe) with off[x] <= g0
  int64_t lo = xb, hi = xe;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= g0) lo = mid;
    else hi = mid;
  }
  out2[0] = lo;
  // smallest x in [xb, xe] with off[x] >= g1
  int64_t a = xb, b = xe;
  while (a < b) {
    int64_t mid = (a + b) >> 1;
    if (off[mid] < g1) a = mid + 1;
    else b = mid;
  }
  out2[1] = a;
}

__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ off, int64_t lo, int64_t hi, int64_t e) {
  // largest x in [lo, hi) with off[x] - off[lo] <= e
  int64_t base = off[lo];
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (off[mid] - base <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Each element of either list finds its row, then its rank in the other
// list of the same row (the two lists hold disjoint z sets).
__global__ void k_merge_write(int64_t x_lo, int64_t x_hi, const int64_t* __restrict__ off_a,
                              const int64_t* __restrict__ off_b, const int64_t* __restrict__ off_out,
                              const int32_t* __restrict__ la, const int32_t* __restrict__ lb, int64_t na, int64_t nb,
                              const int32_t* __restrict__ vals_x, const int32_t* __restrict__ vals_z, int64_t g0,
                              int64_t g1, int32_t* __restrict__ out_x, int32_t* __restrict__ out_z) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < na + nb; e += int64_t(gridDim.x) * blockDim.x) {
    const bool in_a = e < na;
    const int64_t i = in_a ? e : e - na;
    const int64_t* off_s = in_a ? off_a : off_b;
    const int64_t* off_o = in_a ? off_b : off_a;
    const int32_t* ls = in_a ? la : lb;
    const int32_t* lo_ = in_a ? lb : la;
    const int64_t x = row_of(off_s, x_lo, x_hi, i);
    const int64_t rs = off_s[x] - off_s[x_lo];
    const int32_t z = ls[i];
    int64_t rank = i - rs;
    if (lo_) {
      const int64_t o0 = off_o[x] - off_o[x_lo], o1 = off_o[x + 1] - off_o[x_lo];
      rank += lower_bound_dev<int32_t>(lo_, o0, o1, z) - o0;
    }
    const int64_t g = off_out[x] + rank;
    if (g >= g0 && g < g1) {
      out_x[g - g0] = vals_x[x];
      out_z[g - g0] = vals_z[z];
    }
  }
}

__global__ void k_gather_values(const int32_t* __restrict__ vals, const int32_t* __restrict__ idx, int64_t n,
                                int32_t* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    out[i] = vals[idx[i]];
}

// digest term of a pair: mix64 of its order-preserving key (both values
// sign-flipped, x in the high word)
__device__ __forceinline__ uint64_t pair_mix(int32_t x, int32_t z) {
  return mix64((uint64_t(uint32_t(x) ^ 0x80000000u) << 32) | uint64_t(uint32_t(z) ^ 0x80000000u));
}

// acc += sum of pair_mix over the n pairs (wrapping): one 64-bit atomic per wave
__global__ void k_digest_pairs(const int32_t* __restrict__ x, const int32_t* __restrict__ z, int64_t n,
                               unsigned long long* __restrict__ acc) {
  uint64_t d = 0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    d += pair_mix(x[i], z[i]);
  d = wave_sum(d);
  if (lane_id() == 0 && d != 0) atomicAdd(acc, (unsigned long long)d);
}

}  // namespace

void digest_pairs(const int32_t* x, const int32_t* z, int64_t n, uint64_t* acc, hipStream_t s) {
  if (n <= 0) return;
  const int grid = int(std::min<int64_t>((n + NT * 8 - 1) / (NT * 8), 4096));
  hipLaunchKernelGGL(k_digest_pairs, dim3(grid), dim3(NT), 0, s, x, z, n,
                     reinterpret_cast<unsigned long long*>(acc));
  JP_LAUNCH_CHECK();
}

void gather_values(const int32_t* vals, const int32_t* idx, int64_t n, int32_t* out, hipStream_t s) {
  if (n <= 0) return;
  int g = int(std::min<int64_t>((n + NT - 1) / NT, 1 << 16));
  hipLaunchKernelGGL(k_gather_values, dim3(g), dim3(NT), 0, s, vals, idx, n, out);
  JP_LAUNCH_CHECK();
}

void add_counts(const int32_t* a, const int32_t* b, int64_t n, int32_t* out, hipStream_t s) {
  if (n <= 0) return;
  int g = int(std::min<int64_t>((n + NT - 1) / NT, 1 << 16));
  hipLaunchKernelGGL(k_add_counts, dim3(g), dim3(NT), 0, s, a, b, n, out);
  JP_LAUNCH_CHECK();
}

void inst_sums(const int32_t* cnt_sp, const int32_t* cnt_de, const int32_t* x_base, int n_inst, int64_t n_x,
               int64_t* tot, hipStream_t s) {
  fill_i64(tot, 3 * int64_t(n_inst), 0, s);
  if (n_x <= 0) return;
  hipLaunchKernelGGL(k_inst_sums, dim3(chunk_grid(n_x)), dim3(NT), 0, s, cnt_sp, cnt_de, x_base, n_inst, n_x, tot);
  JP_LAUNCH_CHECK();
}

void find_rows(const int64_t* off, int64_t x_begin, int64_t x_end, int64_t g0, int64_t g1, int64_t* out2,
               hipStream_t s) {
  hipLaunchKernelGGL(k_find_rows, dim3(1), dim3(64), 0, s, off, x_begin, x_end, g0, g1, out2);
  JP_LAUNCH_CHECK();
}

void merge_write_n(int64_t x_lo, int64_t x_hi, const int64_t* off_a, const int64_t* off_b, const int64_t* off_out,
                   const int32_t* la, const int32_t* lb, int64_t na, int64_t nb, const int32_t* vals_x,
                   const int32_t* vals_z, int64_t g0, int64_t g1, int32_t* out_x, int32_t* out_z, hipStream_t s) {
  int64_t n = na + nb;
  if (n <= 0) return;
  int g = int(std::min<int64_t>((n + NT - 1) / NT, 1 << 16));
  hipLaunchKernelGGL(k_merge_write, dim3(g), dim3(NT), 0, s, x_lo, x_hi, off_a, off_b, off_out, la, lb, na, nb, vals_x,
                     vals_z, g0, g1, out_x, out_z);
  JP_LAUNCH_CHECK();
}

}  // namespace jp
