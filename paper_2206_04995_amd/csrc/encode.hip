// Dictionary encoding of multi-column keys (paper Sec. 2.2, "Supporting Wider
// Range of Join-Project Operations"): a tuple of attributes is mapped to one
// consecutive natural number, so a Join-Project whose x, y or z is a tuple of
// columns runs as the single-column operation over the ids.
//
// The ids are the ranks of the distinct tuples in lexicographic order (each
// column compared as signed int32), so id order is tuple order and a result
// sorted by ids is sorted by tuples.  Several parts (say R.y and S.y, whose
// ids must agree for the join) are encoded together.  The rows of all parts
// are sorted by an LSD pass per column (last column first, each a stable
// radix sort of the column's values in the order left by the previous pass);
// a row starts a new id where any column differs from its predecessor.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/jp.h"
#include "common.h"
#include "plan_impl.h"
#include "pool.h"
#include "prim.h"

struct jp_dict {
  jp::Budget B;
  jp::Arena A{&B};
  int32_t n_cols = 0;
  int64_t n_distinct = 0;
  std::vector<int32_t*> vals;  // per column: the distinct tuples' values, in id order
};

namespace {

using namespace jp;

constexpr int NT = 256;
constexpr int MAX_COLS = 8;

inline int grid(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + NT - 1) / NT, 1 << 20))); }

#define GRID_STRIDE(i, n) \
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < (n); i += int64_t(gridDim.x) * blockDim.x)

__global__ void k_iota(uint32_t* __restrict__ p, int64_t n) {
  GRID_STRIDE(i, n) { p[i] = uint32_t(i); }
}

// keys[i] = col[perm[i]] - mn (perm null: identity), as an unsigned offset
__global__ void k_col_keys(const int32_t* __restrict__ col, const uint32_t* __restrict__ perm, int64_t n, int32_t mn,
                           uint32_t* __restrict__ keys) {
  GRID_STRIDE(i, n) {
    const int32_t v = col[perm ? perm[i] : i];
    keys[i] = uint32_t(int64_t(v) - int64_t(mn));
  }
}

struct Cols {
  const int32_t* c[MAX_COLS];
  int n;
};

// flags[i] = 1 iff sorted row i differs from sorted row i - 1 in some column
__global__ void k_tuple_heads(Cols cols, const uint32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ flags) {
  GRID_STRIDE(i, n) {
    int f = i == 0 ? 1 : 0;
    if (!f) {
      const uint32_t a = perm[i], b = perm[i - 1];
      for (int c = 0; c < cols.n; ++c)
        if (cols.c[c][a] != cols.c[c][b]) {
          f = 1;
          break;
        }
    }
    flags[i] = f;
  }
}

struct OutCols {
  int32_t* c[MAX_COLS];
  int n;
};

// ids[perm[i]] = rank of sorted row i; the first row of each id writes its tuple
__global__ void k_tuple_ids(Cols cols, const uint32_t* __restrict__ perm, const int32_t* __restrict__ flags,
                            const int32_t* __restrict__ E, int64_t n, int32_t* __restrict__ ids, OutCols vals) {
  GRID_STRIDE(i, n) {
    const int32_t id = E[i + 1] - 1;
    const uint32_t r = perm[i];
    ids[r] = id;
    if (flags[i])
      for (int c = 0; c < cols.n; ++c) vals.c[c][id] = cols.c[c][r];
  }
}

// out[c][i] = vals[c][ids[i]]; an id outside [0, nd) sets *bad and writes nothing
__global__ void k_tuple_decode(const int32_t* __restrict__ ids, int64_t n, Cols vals, int64_t nd, OutCols out,
                               int32_t* __restrict__ bad) {
  GRID_STRIDE(i, n) {
    const int32_t id = ids[i];
    if (id < 0 || int64_t(id) >= nd) {
      *bad = 1;
      continue;
    }
    for (int c = 0; c < vals.n; ++c) out.c[c][i] = vals.c[c][id];
  }
}

void launch_check() { JP_LAUNCH_CHECK(); }

jp_status dfail(int st, const std::string& m) {
  set_last_error(m);
  return jp_status(st);
}

template <class F>
jp_status dguard(F&& f) {
  try {
    f();
    return JP_OK;
  } catch (const Error& e) {
    return dfail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return dfail(JP_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return dfail(JP_EHIP, e.what());
  }
}

void build_dict(jp_dict* d, int32_t n_cols, int32_t n_parts, const int32_t* const* cols, const int64_t* n,
                int32_t* const* ids, hipStream_t s) {
  Arena T(&d->B);
  int64_t N = 0;
  for (int p = 0; p < n_parts; ++p) N += n[p];
  // columns of all parts back to back
  std::vector<int32_t*> cat(n_cols);
  for (int c = 0; c < n_cols; ++c) {
    cat[c] = T.alloc<int32_t>(N, s);
    int64_t at = 0;
    for (int p = 0; p < n_parts; ++p) {
      if (n[p]) JP_HIP(hipMemcpyAsync(cat[c] + at, cols[size_t(p) * n_cols + c], n[p] * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, s));
      at += n[p];
    }
  }
  // per-column value ranges (radix sorts take only the bits they span)
  int32_t* base = T.alloc<int32_t>(2, s);
  const int32_t hb[2] = {0, int32_t(N)};
  JP_HIP(hipMemcpyAsync(base, hb, sizeof(hb), hipMemcpyHostToDevice, s));
  int32_t* mm = T.alloc<int32_t>(2 * int64_t(n_cols), s);
  for (int c = 0; c < n_cols; ++c) seg_minmax(cat[c], N, base, 1, mm + 2 * c, mm + 2 * c + 1, s);
  std::vector<int32_t> hmm(2 * size_t(n_cols));
  JP_HIP(hipMemcpyAsync(hmm.data(), mm, hmm.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));

  // LSD over the columns: stable sorts of the row indices, last column first
  uint32_t* perm = T.alloc<uint32_t>(N, s);
  uint32_t* perm2 = T.alloc<uint32_t>(N, s);
  uint32_t* keys = T.alloc<uint32_t>(N, s);
  uint32_t* keys2 = T.alloc<uint32_t>(N, s);
  hipLaunchKernelGGL(k_iota, dim3(grid(N)), dim3(NT), 0, s, perm, N);
  launch_check();
  for (int c = n_cols - 1; c >= 0; --c) {
    const int32_t mn = hmm[2 * c], mx = hmm[2 * c + 1];
    if (mn >= mx) continue;  // one value (or none): the order is unchanged
    hipLaunchKernelGGL(k_col_keys, dim3(grid(N)), dim3(NT), 0, s, cat[c], perm, N, mn, keys);
    launch_check();
    const int bits = bits_for(uint64_t(int64_t(mx) - int64_t(mn) + 1));
    if (radix_sort_pairs(keys, perm, keys2, perm2, N, bits, s, T)) std::swap(perm, perm2);
  }
  Cols cc{};
  cc.n = n_cols;
  for (int c = 0; c < n_cols; ++c) cc.c[c] = cat[c];
  int32_t* flags = T.alloc<int32_t>(N, s);
  hipLaunchKernelGGL(k_tuple_heads, dim3(grid(N)), dim3(NT), 0, s, cc, perm, N, flags);
  launch_check();
  int32_t* E = T.alloc<int32_t>(N + 1, s);
  scan_excl_i32(flags, E, N, s, T);
  int32_t nd = 0;
  JP_HIP(hipMemcpyAsync(&nd, E + N, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  JP_HIP(hipStreamSynchronize(s));
  d->n_distinct = nd;
  d->vals.assign(n_cols, nullptr);
  OutCols oc{};
  oc.n = n_cols;
  for (int c = 0; c < n_cols; ++c) oc.c[c] = d->vals[c] = d->A.alloc<int32_t>(std::max<int64_t>(nd, 1), s);
  int32_t* ids_all = T.alloc<int32_t>(N, s);
  hipLaunchKernelGGL(k_tuple_ids, dim3(grid(N)), dim3(NT), 0, s, cc, perm, flags, E, N, ids_all, oc);
  launch_check();
  int64_t at = 0;
  for (int p = 0; p < n_parts; ++p) {
    if (n[p] && ids[p])
      JP_HIP(hipMemcpyAsync(ids[p], ids_all + at, n[p] * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    at += n[p];
  }
  T.release(s);
  JP_HIP(hipStreamSynchronize(s));
}

}  // namespace

extern "C" {

jp_status jp_dict_create(int32_t n_cols, int32_t n_parts, const int32_t* const* cols, const int64_t* n,
                         int32_t* const* ids, hipStream_t stream, jp_dict** out) {
  if (!out) return dfail(JP_EINVAL, "out is null");
  *out = nullptr;
  if (n_cols < 1 || n_cols > MAX_COLS) return dfail(JP_EINVAL, "n_cols must be in [1, 8]");
  if (n_parts < 1 || !cols || !n || !ids) return dfail(JP_EINVAL, "null argument or no part");
  int64_t N = 0;
  for (int p = 0; p < n_parts; ++p) {
    if (n[p] < 0) return dfail(JP_EINVAL, "negative row count");
    if (n[p] > 0) {
      if (!ids[p]) return dfail(JP_EINVAL, "null id output for a non-empty part");
      for (int c = 0; c < n_cols; ++c)
        if (!cols[size_t(p) * n_cols + c]) return dfail(JP_EINVAL, "null column for a non-empty part");
    }
    N += n[p];
  }
  if (N > INT32_MAX) return dfail(JP_EINVAL, "more than 2^31 - 1 rows over all parts");
  jp_dict* d = new (std::nothrow) jp_dict();
  if (!d) return dfail(JP_ENOMEM, "host allocation failed");
  d->n_cols = n_cols;
  jp_status st = dguard([&] {
    if (N > 0) build_dict(d, n_cols, n_parts, cols, n, ids, stream);
  });
  if (st != JP_OK) {
    delete d;
    return st;
  }
  *out = d;
  return JP_OK;
}

jp_status jp_dict_size(const jp_dict* d, int64_t* n_distinct) {
  if (!d || !n_distinct) return dfail(JP_EINVAL, "null argument");
  *n_distinct = d->n_distinct;
  return JP_OK;
}

jp_status jp_dict_decode(const jp_dict* d, const int32_t* ids, int64_t n, int32_t* const* cols_out,
                         hipStream_t stream) {
  if (!d || !cols_out) return dfail(JP_EINVAL, "null argument");
  if (n < 0) return dfail(JP_EINVAL, "negative count");
  if (n == 0) return JP_OK;
  if (!ids) return dfail(JP_EINVAL, "null ids");
  for (int c = 0; c < d->n_cols; ++c)
    if (!cols_out[c]) return dfail(JP_EINVAL, "null output column");
  if (d->n_distinct == 0) return dfail(JP_ERANGE, "the dictionary is empty");
  return dguard([&] {
    Arena T;
    int32_t* bad = T.alloc<int32_t>(1, stream);
    fill_i32(bad, 1, 0, stream);
    Cols vc{};
    OutCols oc{};
    vc.n = oc.n = d->n_cols;
    for (int c = 0; c < d->n_cols; ++c) {
      vc.c[c] = d->vals[c];
      oc.c[c] = cols_out[c];
    }
    hipLaunchKernelGGL(k_tuple_decode, dim3(grid(n)), dim3(NT), 0, stream, ids, n, vc, d->n_distinct, oc, bad);
    launch_check();
    int32_t hbad = 0;
    JP_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    JP_HIP(hipStreamSynchronize(stream));
    T.release(stream);
    if (hbad) throw Error(JP_ERANGE, "an id lies outside the dictionary");
  });
}

void jp_dict_destroy(jp_dict* d) {
  if (!d) return;
  d->A.release(nullptr);
  delete d;
}

}  // extern "C"
