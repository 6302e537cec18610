// CPU oracle for the Join-Project  PI_{x,z}( R(x,y) JOIN_y S(z,y) ).
//
// TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
// benchmark's CPU-baseline leg may load this library.  It shares no code,
// header or table with the GPU path.
//
// What it computes is the plain definition of the operation (Sec. 1, Eq. 1 of
// the paper): the set of (x, z) such that some y has (x, y) in R and (z, y) in
// S, with the projection removing duplicates.  It follows the paper's
// "classical solution" (Sec. 1.1): a hash join with S as the build side,
// followed by hash-set deduplication of the projected join rows.  The output
// is ordered lexicographically by (x, z) as signed int32; input tuples may
// repeat (set semantics).  The bag join size OUT_J counts every matching
// (R tuple, S tuple) pair, repeats included.
//
// The order-independent digest of a pair set is the wrapping 64-bit sum of
// mix64(key(x, z)), where key flips the sign bit of both values and places x
// in the high word, and mix64 is the SplitMix64 output finaliser
// (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014, with the constants published by Vigna for splitmix64).
//
// Threads split R by ranges of x value; ranges are disjoint, so their result
// sets are disjoint and concatenate in order.
//
// jpo_row_counts reaches the same set through the matrix form of Sec. 1.1
// ((x, z) is in the result iff row x of the Boolean product R S has a 1 at z),
// one x row at a time as a bit vector over the distinct z values.  It keeps
// memory at |Z| bits per thread, so it counts and digests results that are
// far too large to hold in a hash set.

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace {

typedef std::unordered_map<int32_t, std::vector<int32_t>> YIndex;

inline uint64_t pair_key(int32_t x, int32_t z) {
  return (uint64_t(uint32_t(x) ^ 0x80000000u) << 32) | uint64_t(uint32_t(z) ^ 0x80000000u);
}
inline int32_t key_x(uint64_t k) { return int32_t(uint32_t(k >> 32) ^ 0x80000000u); }
inline int32_t key_z(uint64_t k) { return int32_t(uint32_t(k) ^ 0x80000000u); }

inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// Step 1 of the classical solution: hash S on the join key y.
YIndex build_index(const int32_t* sz, const int32_t* sy, int64_t ns) {
  YIndex h;
  h.reserve(size_t(ns / 4 + 16));
  for (int64_t i = 0; i < ns; ++i) h[sy[i]].push_back(sz[i]);
  return h;
}

struct Slices {
  int64_t lo = 0, width = 1;
  int n = 1;
  int of(int32_t x) const {
    int64_t s = (int64_t(x) - lo) / width;
    return int(s);
  }
};

Slices make_slices(const int32_t* rx, int64_t nr, int want) {
  Slices sl;
  if (nr == 0) return sl;
  int32_t mn = rx[0], mx = rx[0];
  for (int64_t i = 1; i < nr; ++i) {
    mn = std::min(mn, rx[i]);
    mx = std::max(mx, rx[i]);
  }
  int64_t range = int64_t(mx) - int64_t(mn) + 1;
  int n = std::max(1, want);
  if (range < n) n = int(range);
  sl.lo = mn;
  sl.width = (range + n - 1) / n;
  sl.n = int((range + sl.width - 1) / sl.width);
  return sl;
}

// R tuple indices grouped by slice.
std::vector<std::vector<int64_t>> bucket_rows(const int32_t* rx, int64_t nr, const Slices& sl) {
  std::vector<std::vector<int64_t>> b(sl.n);
  for (int64_t i = 0; i < nr; ++i) b[sl.of(rx[i])].push_back(i);
  return b;
}

// Steps 2-3: probe the index with one slice of R and deduplicate the projected
// rows in a hash set; returns the slice's keys sorted.
std::vector<uint64_t> slice_result(const std::vector<int64_t>& rows, const int32_t* rx,
                                   const int32_t* ry, const YIndex& h) {
  std::unordered_set<uint64_t> out;
  for (int64_t i : rows) {
    auto it = h.find(ry[i]);
    if (it == h.end()) continue;
    for (int32_t z : it->second) out.insert(pair_key(rx[i], z));
  }
  std::vector<uint64_t> v(out.begin(), out.end());
  std::sort(v.begin(), v.end());
  return v;
}

template <class F>
void parallel_for(int n, int nthreads, F&& f) {
  if (nthreads <= 1 || n <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < std::min(nthreads, n); ++t)
    th.emplace_back([&]() {
      for (int i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& t : th) t.join();
}

}  // namespace

extern "C" {

// Bag join size OUT_J = number of (R tuple, S tuple) pairs with equal y.
int64_t jpo_out_j(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz,
                  const int32_t* sy, int64_t ns) {
  (void)rx;
  YIndex h = build_index(sz, sy, ns);
  int64_t total = 0;
  for (int64_t i = 0; i < nr; ++i) {
    auto it = h.find(ry[i]);
    if (it != h.end()) total += int64_t(it->second.size());
  }
  return total;
}

// Distinct-pair count and digest of the whole result.
int64_t jpo_count(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz,
                  const int32_t* sy, int64_t ns, int nthreads, uint64_t* digest) {
  YIndex h = build_index(sz, sy, ns);
  Slices sl = make_slices(rx, nr, std::max(1, nthreads) * 8);
  auto buckets = bucket_rows(rx, nr, sl);
  std::vector<int64_t> cnt(sl.n, 0);
  std::vector<uint64_t> dig(sl.n, 0);
  parallel_for(sl.n, nthreads, [&](int s) {
    std::vector<uint64_t> v = slice_result(buckets[s], rx, ry, h);
    cnt[s] = int64_t(v.size());
    uint64_t d = 0;
    for (uint64_t k : v) d += mix64(k);
    dig[s] = d;
  });
  int64_t c = 0;
  uint64_t d = 0;
  for (int s = 0; s < sl.n; ++s) {
    c += cnt[s];
    d += dig[s];
  }
  if (digest) *digest = d;
  return c;
}

// Full sorted result.  Writes min(count, cap) pairs; returns the count.
int64_t jpo_list(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz,
                 const int32_t* sy, int64_t ns, int nthreads, int32_t* out_x, int32_t* out_z,
                 int64_t cap) {
  YIndex h = build_index(sz, sy, ns);
  Slices sl = make_slices(rx, nr, std::max(1, nthreads) * 8);
  auto buckets = bucket_rows(rx, nr, sl);
  std::vector<std::vector<uint64_t>> res(sl.n);
  parallel_for(sl.n, nthreads, [&](int s) { res[s] = slice_result(buckets[s], rx, ry, h); });
  int64_t pos = 0;
  for (int s = 0; s < sl.n; ++s) {
    for (uint64_t k : res[s]) {
      if (pos < cap) {
        out_x[pos] = key_x(k);
        out_z[pos] = key_z(k);
      }
      ++pos;
    }
  }
  return pos;
}

// Result rows for selected x values: for each xs[i], the sorted distinct z's
// reachable from it.  counts[i] receives the row size; the rows are written
// back to back into out_z (up to cap values).  Returns the total row length.
int64_t jpo_rows(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz,
                 const int32_t* sy, int64_t ns, const int32_t* xs, int64_t nxs, int nthreads,
                 int64_t* counts, int32_t* out_z, int64_t cap) {
  YIndex h = build_index(sz, sy, ns);
  std::unordered_map<int32_t, int64_t> want;
  for (int64_t i = 0; i < nxs; ++i) want.emplace(xs[i], i);
  std::vector<std::vector<int32_t>> ys(nxs);
  for (int64_t i = 0; i < nr; ++i) {
    auto it = want.find(rx[i]);
    if (it != want.end()) ys[it->second].push_back(ry[i]);
  }
  std::vector<std::vector<int32_t>> rows(nxs);
  parallel_for(int(nxs), nthreads, [&](int i) {
    std::unordered_set<int32_t> zs;
    for (int32_t y : ys[i]) {
      auto it = h.find(y);
      if (it == h.end()) continue;
      for (int32_t z : it->second) zs.insert(z);
    }
    rows[i].assign(zs.begin(), zs.end());
    std::sort(rows[i].begin(), rows[i].end());
  });
  int64_t pos = 0;
  for (int64_t i = 0; i < nxs; ++i) {
    counts[i] = int64_t(rows[i].size());
    for (int32_t z : rows[i]) {
      if (pos < cap) out_z[pos] = z;
      ++pos;
    }
  }
  return pos;
}

// Per-row counts and digests by the matrix form of the definition (Sec. 1.1):
// row x of the Boolean product C = R S is the OR, over the join keys y of x,
// of the 0/1 rows S[y] over the distinct z values.  Each x row is built as a
// bit vector over the sorted distinct z values, one x at a time, so memory
// stays at |Z| bits per thread whatever the result size; a pair is counted
// (and its mix64 added to the row's digest) when its bit goes from 0 to 1.
// Rows are the distinct x values of R in ascending order, including those
// with no match (count 0).  xs_out, cnt_out and dig_out must hold nr entries
// (nullable); *digest receives the digest of the whole result.  Returns the
// number of distinct x values; *total receives the number of pairs.
int64_t jpo_row_counts(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz,
                       const int32_t* sy, int64_t ns, int nthreads, int32_t* xs_out, int64_t* cnt_out,
                       uint64_t* dig_out, int64_t* total, uint64_t* digest) {
  // distinct z values, ascending, and each S tuple's index among them
  std::vector<int32_t> zs(sz, sz + ns);
  std::sort(zs.begin(), zs.end());
  zs.erase(std::unique(zs.begin(), zs.end()), zs.end());
  std::unordered_map<int32_t, std::vector<int32_t>> h;  // y -> z indices (S is the build side)
  h.reserve(size_t(ns / 4 + 16));
  for (int64_t j = 0; j < ns; ++j) {
    const int32_t zi = int32_t(std::lower_bound(zs.begin(), zs.end(), sz[j]) - zs.begin());
    h[sy[j]].push_back(zi);
  }
  // R grouped by x (ascending)
  std::vector<std::pair<int32_t, int32_t>> r(static_cast<size_t>(nr));
  for (int64_t i = 0; i < nr; ++i) r[size_t(i)] = {rx[i], ry[i]};
  std::sort(r.begin(), r.end());
  std::vector<int64_t> start;  // first tuple of each distinct x
  for (int64_t i = 0; i < nr; ++i)
    if (i == 0 || r[size_t(i)].first != r[size_t(i - 1)].first) start.push_back(i);
  const int64_t nx = int64_t(start.size());
  start.push_back(nr);
  std::vector<int64_t> cnt(size_t(nx), 0);
  std::vector<uint64_t> dig(size_t(nx), 0);
  const int64_t words = int64_t(zs.size() / 64 + 1);
  const int64_t per_task = 64;
  const int n_tasks = int((nx + per_task - 1) / per_task);
  parallel_for(n_tasks, nthreads, [&](int t) {
    std::vector<uint64_t> bits(size_t(words), 0);
    std::vector<int64_t> touched;
    for (int64_t k = int64_t(t) * per_task; k < std::min(nx, int64_t(t + 1) * per_task); ++k) {
      const int32_t x = r[size_t(start[size_t(k)])].first;
      int64_t c = 0;
      uint64_t d = 0;
      for (int64_t i = start[size_t(k)]; i < start[size_t(k + 1)]; ++i) {
        auto it = h.find(r[size_t(i)].second);
        if (it == h.end()) continue;
        for (int32_t zi : it->second) {
          uint64_t& w = bits[size_t(zi >> 6)];
          const uint64_t b = uint64_t(1) << (zi & 63);
          if (w & b) continue;
          if (w == 0) touched.push_back(zi >> 6);
          w |= b;
          ++c;
          d += mix64(pair_key(x, zs[size_t(zi)]));
        }
      }
      for (int64_t wi : touched) bits[size_t(wi)] = 0;
      touched.clear();
      cnt[size_t(k)] = c;
      dig[size_t(k)] = d;
    }
  });
  int64_t tc = 0;
  uint64_t td = 0;
  for (int64_t k = 0; k < nx; ++k) {
    if (xs_out) xs_out[k] = r[size_t(start[size_t(k)])].first;
    if (cnt_out) cnt_out[k] = cnt[size_t(k)];
    if (dig_out) dig_out[k] = dig[size_t(k)];
    tc += cnt[size_t(k)];
    td += dig[size_t(k)];
  }
  if (total) *total = tc;
  if (digest) *digest = td;
  return nx;
}

// Join-Aggregate (Sec. 4.1, group-by attributes from both tables): for every
// group (x, z) of the join rows of R(x, y, v) and S(z, y, u), the number of
// join rows and the sum of v * u (int64, wrapping).  The same hash join as the
// classical solution, with the hash set replaced by a hash map from the pair
// key to its (count, sum).  Groups sorted by (x, z) as signed int32; writes
// min(groups, cap) of them and returns the number of groups.
int64_t jpo_aggregate(const int32_t* rx, const int32_t* ry, const int32_t* rv, int64_t nr, const int32_t* sz,
                      const int32_t* sy, const int32_t* su, int64_t ns, int nthreads, int32_t* out_x,
                      int32_t* out_z, int64_t* out_cnt, int64_t* out_sum, int64_t cap) {
  std::unordered_map<int32_t, std::vector<std::pair<int32_t, int32_t>>> h;  // y -> (z, u)
  h.reserve(size_t(ns / 4 + 16));
  for (int64_t j = 0; j < ns; ++j) h[sy[j]].push_back({sz[j], su[j]});
  Slices sl = make_slices(rx, nr, std::max(1, nthreads) * 8);
  auto buckets = bucket_rows(rx, nr, sl);
  struct Agg {
    int64_t cnt = 0;
    uint64_t sum = 0;
  };
  std::vector<std::vector<std::pair<uint64_t, Agg>>> res(sl.n);
  parallel_for(sl.n, nthreads, [&](int s) {
    std::unordered_map<uint64_t, Agg> m;
    for (int64_t i : buckets[s]) {
      auto it = h.find(ry[i]);
      if (it == h.end()) continue;
      for (const auto& zu : it->second) {
        Agg& a = m[pair_key(rx[i], zu.first)];
        a.cnt += 1;
        a.sum += uint64_t(int64_t(rv[i]) * int64_t(zu.second));
      }
    }
    res[s].assign(m.begin(), m.end());
    std::sort(res[s].begin(), res[s].end(),
              [](const std::pair<uint64_t, Agg>& a, const std::pair<uint64_t, Agg>& b) { return a.first < b.first; });
  });
  int64_t pos = 0;
  for (int s = 0; s < sl.n; ++s) {
    for (const auto& e : res[s]) {
      if (pos < cap) {
        out_x[pos] = key_x(e.first);
        out_z[pos] = key_z(e.first);
        out_cnt[pos] = e.second.cnt;
        out_sum[pos] = int64_t(e.second.sum);
      }
      ++pos;
    }
  }
  return pos;
}

// Digest of an explicit pair list (used to digest a listed result).
uint64_t jpo_digest_pairs(const int32_t* xs, const int32_t* zs, int64_t n) {
  uint64_t d = 0;
  for (int64_t i = 0; i < n; ++i) d += mix64(pair_key(xs[i], zs[i]));
  return d;
}

}  // extern "C"
