// Host orchestration of the Join-Project path (paper Alg. 1) and the C ABI
// declared in include/jp.h.  A single query is a batch of one instance: every
// stage runs as one launch over all instances, whose ids occupy disjoint
// ranges of the global x, y and z id spaces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/jp.h"
#include "classical.h"
#include "common.h"
#include "plan_impl.h"
#include "prim.h"
#include "stages.h"

using namespace jp;

namespace {

thread_local std::string g_last_error;

jp_status fail(int st, const std::string& m) {
  g_last_error = m;
  return jp_status(st);
}

template <class F>
jp_status guarded(F&& f) {
  try {
    f();
    return JP_OK;
  } catch (const Error& e) {
    return fail(e.status, e.what());
  } catch (const std::bad_alloc&) {
    return fail(JP_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(JP_EHIP, e.what());
  }
}

template <class T>
void h2d(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) JP_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
void d2h(T* dst, const T* src, size_t n, hipStream_t s) {
  if (n) JP_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, s));
}
void sync(hipStream_t s) { JP_HIP(hipStreamSynchronize(s)); }

double env_double(const char* name, double dflt) {
  const char* v = std::getenv(name);
  if (!v || !*v) return dflt;
  return std::atof(v);
}

// Per-instance key offsets from per-instance ranges [mn, mx]: instance i's keys
// are koff[i] + (v - mn[i]).  Returns the number of key bits.
int key_layout(const std::vector<int32_t>& mn, const std::vector<int32_t>& mx, std::vector<int64_t>& koff) {
  int n = int(mn.size());
  koff.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    int64_t rng = mn[i] <= mx[i] ? int64_t(mx[i]) - int64_t(mn[i]) + 1 : 0;
    koff[i + 1] = koff[i] + rng;
  }
  if (koff[n] > (int64_t(1) << 32))
    throw Error(JP_EINVAL, "the instances' value ranges add up to more than 2^32 keys; split the batch");
  return bits_for(uint64_t(koff[n]));
}

// key bits of the widest instance range (a segmented sort sorts only these)
int local_bits(const std::vector<int64_t>& koff) {
  int64_t w = 0;
  for (size_t i = 0; i + 1 < koff.size(); ++i) w = std::max<int64_t>(w, koff[i + 1] - koff[i]);
  return bits_for(uint64_t(w));
}

__global__ void k_slice_info(const int64_t* __restrict__ off_de, const int64_t* __restrict__ off_sp,
                             const int64_t* __restrict__ rows, int64_t* __restrict__ info) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int64_t lo = rows[0], hi = rows[1];
    info[0] = lo;
    info[1] = hi;
    info[2] = off_de[lo];
    info[3] = off_de[hi];
    info[4] = off_sp[lo];
    info[5] = off_sp[hi];
  }
}

inline int grid_of(int64_t n) { return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16))); }

}  // namespace

namespace jp {

void set_last_error(const std::string& m) { g_last_error = m; }

// Threshold tau of f2 (paper Sec. 2.6): a z is dense iff T_sparseBMM(z) >
// T_denseEC(z).  With OUT_{J,z} estimated as m_z / |S| * OUT_J (as in the
// paper), T_sparseBMM(z) = c_fix / |Z| + c_sp * m_z / |S| * OUT_J and
// T_denseEC(z) = c_de * |X| (one bit decision per x), so f2 grows with m_z and
// the test is m_z > tau with tau = (c_de |X| - c_fix / |Z|) |S| / (c_sp OUT_J).
int64_t tau_from_cost(int64_t nx, int64_t nz, int64_t ns, int64_t out_j, double c_de_over_sp, double c_fix_over_sp) {
  if (out_j <= 0 || nz <= 0 || nx <= 0) return INT64_MAX;
  double t = (c_de_over_sp * double(nx) - c_fix_over_sp / double(nz)) * double(ns) / double(out_j);
  if (t < -1.0) return -1;
  if (t > 9.0e18) return INT64_MAX;
  return int64_t(std::floor(t));
}

void Plan::build(const jp_instance* inst, int n, const jp_options* o, hipStream_t s) {
  n_inst = n;
  if (o) opt = *o;
  else std::memset(&opt, 0, sizeof(opt));
  stream = s;
  stream_used = true;
  arena_limit(opt.workspace_limit_bytes);
  const bool timing = (opt.flags & JP_FLAG_TIMING) != 0;
  if (timing) {
    for (auto& e : evp) JP_HIP(hipEventCreate(&e));
    JP_HIP(hipEventRecord(evp[0], s));
  }
  h_rbase.assign(n + 1, 0);
  h_sbase.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    h_rbase[i + 1] = h_rbase[i] + int32_t(inst[i].n_r);
    h_sbase[i + 1] = h_sbase[i] + int32_t(inst[i].n_s);
  }
  NR = h_rbase[n];
  NS = h_sbase[n];

  d_rbase = A.alloc<int32_t>(n + 1, s);
  d_sbase = A.alloc<int32_t>(n + 1, s);
  h2d(d_rbase, h_rbase.data(), n + 1, s);
  h2d(d_sbase, h_sbase.data(), n + 1, s);

  if (n == 1) {
    rx = inst[0].r_x;
    ry = inst[0].r_y;
    sz = inst[0].s_z;
    sy = inst[0].s_y;
  } else {
    std::vector<const int32_t*> ptrs(4 * size_t(n));
    for (int i = 0; i < n; ++i) {
      ptrs[i] = inst[i].r_x;
      ptrs[n + i] = inst[i].r_y;
      ptrs[2 * n + i] = inst[i].s_z;
      ptrs[3 * n + i] = inst[i].s_y;
    }
    const int32_t** d_ptrs = A.alloc<const int32_t*>(4 * int64_t(n), s);
    h2d(d_ptrs, ptrs.data(), ptrs.size(), s);
    // per-instance min and max of z, y (S) and x (R): the mapping's key layouts
    d_minmax = A.alloc<int32_t>(6 * int64_t(n), s);
    int32_t *zmin = d_minmax, *zmax = d_minmax + n, *ymin = d_minmax + 2 * n, *ymax = d_minmax + 3 * n;
    int32_t *xmin = d_minmax + 4 * n, *xmax = d_minmax + 5 * n;
    fill_minmax(d_minmax, n, s);
    const int32_t* const* src = d_ptrs;
    // The sort path reads the instances' columns in place (the z sort's first
    // pass and the semi-join take one buffer per instance), so only the min and
    // max are taken here.  The direct-range mapping and the f1 sample read one
    // concatenated buffer per column, which the same pass fills.
    const bool in_place = (opt.flags & JP_FLAG_DIRECT_IDS) == 0 && !f1_probe;
    if (in_place) {
      d_cols = src;
      gather_cols(src, d_rbase, n, NR, nullptr, xmin, xmax, s);
      gather_cols(src + 2 * n, d_sbase, n, NS, nullptr, zmin, zmax, s);
      gather_cols(src + 3 * n, d_sbase, n, NS, nullptr, ymin, ymax, s);
    } else {
      int32_t* cat = A.alloc<int32_t>(2 * NR + 2 * NS, s);
      int32_t *crx = cat, *cry = cat + NR, *csz = cat + 2 * NR, *csy = cat + 2 * NR + NS;
      gather_cols(src, d_rbase, n, NR, crx, xmin, xmax, s);
      gather_cols(src + n, d_rbase, n, NR, cry, nullptr, nullptr, s);
      gather_cols(src + 2 * n, d_sbase, n, NS, csz, zmin, zmax, s);
      gather_cols(src + 3 * n, d_sbase, n, NS, csy, ymin, ymax, s);
      rx = crx;
      ry = cry;
      sz = csz;
      sy = csy;
    }
  }
  map(s);
  if (take_classical) return;  // f1 chose the classical path: the caller builds it
  if (timing) JP_HIP(hipEventRecord(evp[1], s));
  partition(s);
  if (timing) JP_HIP(hipEventRecord(evp[2], s));
}

// ---------------------------------------------------------------- mapping
// With JP_FLAG_DIRECT_IDS, a key space of at most this many keys per column
// element is mapped directly (key histogram, scans, scatter) instead of by
// radix sort.
constexpr int64_t DIRECT_KEYS_PER_ELEM = 2;
constexpr int64_t DIRECT_KEYS_SLACK = 65536;

// Key offsets as key_layout, without its limit: returns koff[n] (the key space).
int64_t key_space(const std::vector<int32_t>& mn, const std::vector<int32_t>& mx, std::vector<int64_t>& koff) {
  const int n = int(mn.size());
  koff.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) koff[i + 1] = koff[i] + (mn[i] <= mx[i] ? int64_t(mx[i]) - int64_t(mn[i]) + 1 : 0);
  return koff[n];
}

bool direct_ok(int64_t keys, int64_t n_elem) {
  return keys <= DIRECT_KEYS_PER_ELEM * n_elem + DIRECT_KEYS_SLACK && keys < (int64_t(1) << 31) - 1;
}

void Plan::map(hipStream_t s) {
  const int n = n_inst;
  Arena T(&B);  // temporaries of the mapping stage
  const bool sort_ids = (opt.flags & JP_FLAG_DIRECT_IDS) == 0;
  // per-instance min and max of S.z, S.y and R.x (all of R: the x keys' layout); a batch's gather took them
  int32_t* mm = d_minmax ? d_minmax : T.alloc<int32_t>(6 * int64_t(n), s);
  int32_t *zmin = mm, *zmax = mm + n, *ymin = mm + 2 * n, *ymax = mm + 3 * n, *xmin = mm + 4 * n, *xmax = mm + 5 * n;
  if (!d_minmax) {
    seg_minmax(sz, NS, d_sbase, n, zmin, zmax, s);
    seg_minmax(sy, NS, d_sbase, n, ymin, ymax, s);
    seg_minmax(rx, NR, d_rbase, n, xmin, xmax, s);
  }
  std::vector<int32_t> h_mm(6 * size_t(n));
  d2h(h_mm.data(), mm, 6 * size_t(n), s);
  // f1 (Sec. 2.6) rides on this first read-back: the classical path when the
  // sampled OUT_J is small against the input
  unsigned long long h_match = 0;
  if (f1_probe) {
    unsigned long long* dm = T.alloc<unsigned long long>(1, s);
    launch_out_j_sample(ry, NR, sy, NS, dm, s);
    d2h(&h_match, dm, 1, s);
  }
  sync(s);
  if (f1_probe && f1_prefers_classical(out_j_from_sample(h_match, NR, NS), NR, NS)) {
    take_classical = true;
    T.release(s);
    return;
  }
  auto part = [&](int k) { return std::vector<int32_t>(h_mm.begin() + k * n, h_mm.begin() + (k + 1) * n); };
  std::vector<int64_t> koff_z, koff_y, koff_x;
  int zbits = key_layout(part(0), part(1), koff_z);
  int ybits = key_layout(part(2), part(3), koff_y);
  const bool direct_z = !sort_ids && direct_ok(koff_z[n], NS);
  bool direct_x = false;
  if (!sort_ids) direct_x = direct_ok(key_space(part(4), part(5), koff_x), NR);
  const int xbits = direct_x ? 0 : key_layout(part(4), part(5), koff_x);
  int64_t* d_koff = T.alloc<int64_t>(3 * (int64_t(n) + 1), s);
  int64_t *dkz = d_koff, *dky = d_koff + (n + 1), *dkx = d_koff + 2 * (n + 1);
  h2d(dkz, koff_z.data(), n + 1, s);
  h2d(dky, koff_y.data(), n + 1, s);
  h2d(dkx, koff_x.data(), n + 1, s);
  map_direct = (direct_z ? 1 : 0) | (direct_x ? 2 : 0);

  const int64_t NSa = std::max<int64_t>(NS, 1);
  uint32_t* k1 = T.alloc<uint32_t>(NSa, s);
  uint32_t* v1 = T.alloc<uint32_t>(NSa, s);
  uint32_t* k2 = T.alloc<uint32_t>(NSa, s);
  uint32_t* v2 = T.alloc<uint32_t>(NSa, s);
  int32_t* d_counts = T.alloc<int32_t>(4, s);

  // z ids and m_z; then S in z order with its y keys and z ids (yk, yp) ready
  // for the stable sort by y.  The sort ping-pongs between (yk, yp) and
  // (ok, op); its pass count is known here, so the buffer its z ids end in is
  // scol itself (no copy afterwards).
  const int ybits_sort = n > 1 ? local_bits(koff_y) : ybits;
  const bool y_odd = radix_passes(NS, ybits_sort) & 1;
  scol = A.alloc<int32_t>(NSa, s);
  uint32_t* const scol_u = reinterpret_cast<uint32_t*>(scol);
  uint32_t *yk, *yp, *ok, *op;
  vals_z = A.alloc<int32_t>(NSa, s);
  z_base = A.alloc<int32_t>(n + 1, s);
  if (direct_z) {
    const int64_t K = koff_z[n];
    int32_t* cnt = T.alloc<int32_t>(K + 1, s);
    fill_i32(cnt, K + 1, 0, s);
    key_hist(sz, NS, d_sbase, n, dkz, zmin, nullptr, cnt, s);
    int32_t* pres = T.alloc<int32_t>(std::max<int64_t>(K, 1), s);
    presence(cnt, K, pres, s);
    int32_t* Ezk = T.alloc<int32_t>(K + 1, s);
    scan_excl_i32(pres, Ezk, K, s, T);
    int32_t* Czk = T.alloc<int32_t>(K + 1, s);
    scan_excl_i32(cnt, Czk, K, s, T);
    m_z = A.alloc<int32_t>(std::max<int64_t>(std::min(K, NS), 1), s);
    key_ids(cnt, K, Ezk, Czk, dkz, zmin, n, vals_z, m_z, nullptr, s);
    bases_from_koff(Ezk, dkz, n, z_base, s);
    yk = k1;
    yp = y_odd ? v1 : scol_u;
    ok = k2;
    op = y_odd ? scol_u : v2;
    scatter_z(sz, sy, NS, d_sbase, n, dkz, zmin, dky, ymin, Ezk, Czk, yk, yp, s);
    JP_HIP(hipMemcpyAsync(d_counts + 0, Ezk + K, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  } else {
    // S sorted by (instance, z): z ids, m_z.  The sort's first pass makes the
    // z keys as it reads S.z; S.y rides along.
    const SortSegments sseg_z{n, d_sbase, dkz, h_sbase};
    const int zbits_sort = n > 1 ? local_bits(koff_z) : zbits;
    bool alt = false;
    if (radix_passes(NS, zbits_sort) > 0) {
      alt = radix_sort_raw(sz, sy, d_cols ? d_cols + 2 * n : nullptr, d_cols ? d_cols + 3 * n : nullptr, zmin, k1, v1,
                           k2, v2, NS, zbits_sort, s, T, sseg_z);
    } else {
      const int32_t *zc = sz, *yc = sy;
      if (d_cols) {  // no sort pass to read the instances' buffers: concatenate them for the key pass
        int32_t* tz = T.alloc<int32_t>(NSa, s);
        int32_t* ty = T.alloc<int32_t>(NSa, s);
        gather_cols(d_cols + 2 * n, d_sbase, n, NS, tz, nullptr, nullptr, s);
        gather_cols(d_cols + 3 * n, d_sbase, n, NS, ty, nullptr, nullptr, s);
        zc = tz;
        yc = ty;
      }
      make_keys(zc, NS, d_sbase, n, dkz, zmin, k1, v1, yc, s);
    }
    uint32_t *zk = alt ? k2 : k1, *zp = alt ? v2 : v1;
    // z ids of the sorted positions go straight into the y sort's input, with
    // the carried S.y as its keys
    zfirst = A.alloc<int32_t>(NS + 1, s);
    yk = alt ? k1 : k2;  // the free pair
    yp = y_odd ? (alt ? v1 : v2) : scol_u;
    const RunCarry carry{reinterpret_cast<const int32_t*>(zp), dky, ymin, yk, yp};
    run_ids(zk, NS, dkz, zmin, n, nullptr, zfirst, vals_z, s, T, d_counts + 0, &carry);
    ids_at_bases(zfirst, d_counts + 0, d_sbase, n, z_base, s);
    ok = zk;  // reuse the z-sorted pair as scratch
    op = y_odd ? scol_u : zp;
  }

  // S sorted by (instance, y), z ascending inside each y: CSR of S by y
  const SortSegments sseg_y{n, d_sbase, dky, h_sbase};
  bool alt2 = radix_sort_pairs(yk, yp, ok, op, NS, ybits_sort, s, T, &sseg_y);
  uint32_t* syk = alt2 ? ok : yk;
  if ((alt2 ? op : yp) != scol_u) throw Error(JP_EHIP, "radix sort pass count differs from its plan");
  Ey = A.alloc<int32_t>(NS + 1, s);
  sptr = A.alloc<int32_t>(NS + 1, s);
  vals_y = A.alloc<int32_t>(NSa, s);
  // the semi-join's y table (dense key domain: a table lookup instead of a
  // binary search); on the sort path the y run ids fill it at their run heads
  const int64_t y_keys = koff_y[n];
  const bool y_table = y_keys <= 2 * NS + 65536;
  int32_t* table = y_table ? T.alloc<int32_t>(std::max<int64_t>(y_keys, 1), s) : nullptr;
  const bool table_by_runs = y_table && !direct_x;
  if (table_by_runs) fill_i32(table, y_keys, -1, s);
  run_ids(syk, NS, dky, ymin, n, Ey, sptr, vals_y, s, T, d_counts + 1, nullptr, table_by_runs ? table : nullptr);
  y_base = A.alloc<int32_t>(n + 1, s);
  gather_bases(Ey, d_sbase, n, y_base, s);

  // semi-join of R on S.y (Sec. 2.2, optimisation 2), then R' grouped by (instance, x)
  const int64_t NRa = std::max<int64_t>(NR, 1);
  d_rpbase = A.alloc<int32_t>(n + 1, s);
  h_rpbase.resize(n + 1);
  int32_t counts[4];
  x_base = A.alloc<int32_t>(n + 1, s);
  if (direct_x) {
    int32_t* yid = T.alloc<int32_t>(NRa, s);
    int32_t* flags = T.alloc<int32_t>(NRa, s);
    if (y_table)
      semijoin_direct(ry, NR, d_rbase, n, syk, NS, sptr, d_counts + 1, dky, y_keys, ymin, table, flags, yid, s);
    else
      semijoin(ry, NR, d_rbase, n, vals_y, y_base, flags, yid, s);
    // x ids over the kept tuples' keys; R' rows by a scatter with per-key cursors
    const int64_t K = koff_x[n];
    int32_t* cnt = T.alloc<int32_t>(K + 1, s);
    fill_i32(cnt, K + 1, 0, s);
    key_hist(rx, NR, d_rbase, n, dkx, xmin, yid, cnt, s);
    int32_t* pres = T.alloc<int32_t>(std::max<int64_t>(K, 1), s);
    presence(cnt, K, pres, s);
    int32_t* Exk = T.alloc<int32_t>(K + 1, s);
    scan_excl_i32(pres, Exk, K, s, T);
    int32_t* Cxk = T.alloc<int32_t>(K + 1, s);
    scan_excl_i32(cnt, Cxk, K, s, T);
    bases_from_koff(Cxk, dkx, n, d_rpbase, s);
    bases_from_koff(Exk, dkx, n, x_base, s);
    JP_HIP(hipMemcpyAsync(d_counts + 2, Cxk + K, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    JP_HIP(hipMemcpyAsync(d_counts + 3, Exk + K, sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    d2h(counts, d_counts, 4, s);
    d2h(h_rpbase.data(), d_rpbase, n + 1, s);
    sync(s);
    NZ = counts[0];
    NY = counts[1];
    NRp = counts[2];
    NX = counts[3];
    const int64_t NRpa = std::max<int64_t>(NRp, 1);
    rptr = A.alloc<int32_t>(NX + 1, s);
    vals_x = A.alloc<int32_t>(std::max<int64_t>(NX, 1), s);
    key_ids(cnt, K, Exk, Cxk, dkx, xmin, n, vals_x, nullptr, rptr, s);
    rcol = A.alloc<int32_t>(NRpa, s);
    scatter_x(rx, yid, NR, d_rbase, n, dkx, xmin, Cxk, rcol, s);
  } else {
    // kept tuples in order with their x keys and y ids, in one pass
    uint32_t* xk = T.alloc<uint32_t>(NRa, s);
    uint32_t* rpy = T.alloc<uint32_t>(NRa, s);
    const SemiJoinIn sj{rx, ry, d_cols, d_cols ? d_cols + n : nullptr, NR, d_rbase, n, dky, ymin, table, vals_y,
                        y_base, dkx, xmin};
    semijoin_compact(sj, xk, rpy, d_rpbase, d_counts + 2, s, T);
    d2h(counts, d_counts, 3, s);
    d2h(h_rpbase.data(), d_rpbase, n + 1, s);
    sync(s);
    NZ = counts[0];
    NY = counts[1];
    NRp = counts[2];

    const int64_t NRpa = std::max<int64_t>(NRp, 1);
    uint32_t* xk2 = T.alloc<uint32_t>(NRpa, s);
    // with an odd pass count the sorted y ids end in the alternate buffer: rcol itself
    const int xbits_sort = n > 1 ? local_bits(koff_x) : xbits;
    const bool x_odd = radix_passes(NRp, xbits_sort) & 1;
    rcol = A.alloc<int32_t>(NRpa, s);
    uint32_t* xp2 = x_odd ? reinterpret_cast<uint32_t*>(rcol) : T.alloc<uint32_t>(NRpa, s);
    const SortSegments sseg_x{n, d_rpbase, dkx, h_rpbase};
    bool alt3 = radix_sort_pairs(xk, rpy, xk2, xp2, NRp, xbits_sort, s, T, &sseg_x);
    uint32_t *sxk = alt3 ? xk2 : xk, *sxp = alt3 ? xp2 : rpy;
    rptr = A.alloc<int32_t>(NRp + 1, s);
    vals_x = A.alloc<int32_t>(NRpa, s);
    int32_t* d_nx = T.alloc<int32_t>(1, s);
    run_ids(sxk, NRp, dkx, xmin, n, nullptr, rptr, vals_x, s, T, d_nx);
    ids_at_bases(rptr, d_nx, d_rpbase, n, x_base, s);
    if (NRp && sxp != reinterpret_cast<uint32_t*>(rcol))
      JP_HIP(hipMemcpyAsync(rcol, sxp, NRp * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }

  // degree statistics (Sec. 2.6): m_z, d_R(y), d_S(y), OUT_J per instance
  const int64_t NYa = std::max<int64_t>(NY, 1);
  if (!direct_z) {
    m_z = A.alloc<int32_t>(std::max<int64_t>(NZ, 1), s);
    run_lengths(zfirst, NZ, m_z, s);
  }
  dR = A.alloc<int32_t>(NYa, s);
  dS = A.alloc<int32_t>(NYa, s);
  fill_i32(dR, NY, 0, s);
  histogram(reinterpret_cast<const uint32_t*>(rcol), NRp, dR, s, NY);
  run_lengths(sptr, NY, dS, s);
  d_outj = A.alloc<int64_t>(n, s);
  out_j_per_inst(dR, dS, NY, y_base, n, d_outj, s);

  h_xbase.resize(n + 1);
  h_ybase.resize(n + 1);
  h_zbase.resize(n + 1);
  h_outj.resize(n);
  d2h(h_xbase.data(), x_base, n + 1, s);
  d2h(h_ybase.data(), y_base, n + 1, s);
  d2h(h_zbase.data(), z_base, n + 1, s);
  d2h(h_outj.data(), d_outj, n, s);
  sync(s);
  NX = h_xbase[n];
  T.release(s);
}

// -------------------------------------------------------------- partition
void Plan::partition(hipStream_t s) {
  const int n = n_inst;
  Arena T(&B);
  const double c_de = env_double("JP_COST_DE_OVER_SP", 0.05);
  const double c_fix = env_double("JP_COST_FIX_OVER_SP", 0.0);
  h_tau.resize(n);
  h_rec.assign(n, TuneRec{});
  for (int i = 0; i < n; ++i) {
    int64_t nx = h_xbase[i + 1] - h_xbase[i], nz = h_zbase[i + 1] - h_zbase[i];
    int64_t ns = h_sbase[i + 1] - h_sbase[i];
    tuned_record(shape_signature(nx, nz, ns, h_outj[i]), &h_rec[i]);  // stored by jp_tune, if any
    if (opt.tau_mode == JP_TAU_FIXED) {
      h_tau[i] = opt.dense_threshold;
    } else if (h_rec[i].valid) {
      h_tau[i] = tau_from_cost(nx, nz, ns, h_outj[i], h_rec[i].ratio, 0.0);
    } else {
      h_tau[i] = tau_from_cost(nx, nz, ns, h_outj[i], c_de, c_fix);
    }
  }
  d_tau = A.alloc<int64_t>(n, s);
  h2d(d_tau, h_tau.data(), n, s);
  // SparseBMM class bounds and the MFMA tile: pinned by the options, else the first instance's tuned record
  const TuneRec& r0 = h_rec[0];
  light_max = opt.sparse_light_max > 0 ? opt.sparse_light_max : (r0.valid && r0.sparse_light_max > 0 ? r0.sparse_light_max : 1024);
  med_max = opt.sparse_med_max > 0 ? opt.sparse_med_max : (r0.valid && r0.sparse_med_max > 0 ? r0.sparse_med_max : 8192);
  med_max = std::max(med_max, light_max);
  mfma_tile = opt.mfma_tile > 0 ? opt.mfma_tile : (r0.valid ? r0.mfma_tile : 0);

  const int64_t NZa = std::max<int64_t>(NZ, 1), NSa = std::max<int64_t>(NS, 1), NYa = std::max<int64_t>(NY, 1);
  zflag = A.alloc<int32_t>(NZa, s);
  dense_flags(m_z, NZ, z_base, n, d_tau, zflag, s);
  Edz = A.alloc<int32_t>(NZ + 1, s);
  scan_excl_i32(zflag, Edz, NZ, s, T);
  dz2z = A.alloc<int32_t>(NZa, s);
  dense_index(zflag, Edz, NZ, dz2z, s);
  zd_base = A.alloc<int32_t>(n + 1, s);
  gather_bases(Edz, z_base, n, zd_base, s);

  // S_sparse: CSR by y of the entries whose z is sparse
  spcol = A.alloc<int32_t>(NSa, s);  // sized before the count is known: one pass fills it
  spptr = A.alloc<int32_t>(NY + 1, s);
  int32_t* d_nsp = T.alloc<int32_t>(1, s);
  filter_rows(false, Ey, scol, NS, zflag, NZ, nullptr, spcol, nullptr, spptr, NY, d_nsp, s, T);
  int32_t nsp = 0;
  d2h(&nsp, d_nsp, 1, s);
  int32_t* hist = T.alloc<int32_t>(int64_t(n) * 32, s);
  hot_histogram(sptr, spptr, dR, NY, y_base, n, hist, s);
  std::vector<int32_t> h_hist(size_t(n) * 32);
  d2h(h_hist.data(), hist, size_t(n) * 32, s);
  h_zdbase.resize(n + 1);
  d2h(h_zdbase.data(), zd_base, n + 1, s);
  sync(s);
  NSp = nsp;
  NZd = h_zdbase[n];

  DenseSpace& d0 = ds[0];
  d0.h_base = h_zdbase;
  d0.base = zd_base;
  if (NZd == 0) {
    // no dense z in any instance: DenseEC has no work, its tables stay empty
    empty_space(d0, s);
    T.release(s);
    return;
  }
  int32_t* zmap = T.alloc<int32_t>(NZa, s);
  zmap_dense(zflag, Edz, NZ, z_base, zd_base, n, zmap, s);
  build_space(d0, zmap, sptr, spptr, &h_hist, T, s);
  dense_keys0 = 0;  // keys with a dense S entry and an R row (the hot histogram covers them all)
  for (int q = 0; q < 32; ++q) dense_keys0 += h_hist[q];
  choose_dense_kernel(T, s);
  if (!use_mfma) {
    pivot_split(T, s);
    narrow_segments(s);
  }
  T.release(s);
}

void Plan::narrow_segments(hipStream_t s) {
  const DenseSpace& d0 = ds[0];
  const int64_t bound[N_WIDTH_CLASSES + 1] = {0, NARROW_SMALL, NARROW_MID, NARROW_MAX, INT64_MAX};
  for (int k = 0; k < N_WIDTH_CLASSES; ++k) {
    const int64_t lo = bound[k] + 1, hi = bound[k + 1];
    std::vector<int32_t>& x0 = h_nar_x0[k];
    std::vector<int32_t>& base = h_nar_base[k];
    x0.clear();
    base.assign(1, 0);
    for (int i = 0; i < n_inst; ++i) {
      const int64_t zd = d0.h_base[i + 1] - d0.h_base[i], nx = h_xbase[i + 1] - h_xbase[i];
      if (zd >= lo && zd <= hi && nx > 0) {
        x0.push_back(h_xbase[i]);
        base.push_back(base.back() + int32_t(nx));
      }
    }
    nar_m[k] = int(x0.size());
    nar_rows[k] = base.back();
    if (nar_m[k] == 0) continue;
    nar_x0[k] = A.alloc<int32_t>(nar_m[k], s);
    nar_base[k] = A.alloc<int32_t>(nar_m[k] + 1, s);
    h2d(nar_x0[k], x0.data(), x0.size(), s);
    h2d(nar_base[k], base.data(), base.size(), s);
  }
  nar_listed = true;
}

// The count pass of the dense part runs on the INT8 matrix cores when the
// panel of (x, dense key) cells is dense: the product does 2 ops per cell and
// dense z whether or not the cell is set, the bit path one 32-z word per set
// cell (plus its cold scatters), so the product wins when a good share of the
// cells is set.  Single-instance plans only; JP_DENSE_MFMA asks for it
// whenever the panels fit, JP_DENSE_BITS never uses it.
void Plan::choose_dense_kernel(Arena& T, hipStream_t s) {
  use_mfma = false;
  int kernel = opt.dense_kernel;
  if (kernel == JP_DENSE_AUTO && !h_rec.empty() && h_rec[0].valid) kernel = h_rec[0].dense_kernel;  // tuned
  if (n_inst != 1 || kernel == JP_DENSE_BITS || NZd <= 0 || NX <= 0 || dense_keys0 <= 0) return;
  const double min_density = env_double("JP_MFMA_MIN_DENSITY", 1.0 / 32.0);
  if (kernel != JP_DENSE_MFMA && double(NRp) / (double(NX) * double(dense_keys0)) < min_density) return;
  const int64_t NYa = std::max<int64_t>(NY, 1);
  int32_t* kmap = T.alloc<int32_t>(NYa, s);
  K_panel = panel_key_count(sptr, spptr, dR, NY, kmap, T, s);
  if (K_panel <= 0) return;
  k_pad = mfma_pad_keys(K_panel);
  nx_pad = mfma_pad_rows(NX);
  nz_pad = mfma_pad_cols(NZd);
  const int64_t lim = int64_t(1) << 31;
  if (nx_pad * k_pad > lim || nz_pad * k_pad > lim) return;

  use_mfma = true;
  d_mfma_steps = A.alloc<int64_t>(1, s);
  pA = A.alloc<int8_t>(nx_pad * k_pad, s);
  pBt = A.alloc<int8_t>(nz_pad * k_pad, s);
  build_panels(rptr, rcol, NX, Ey, scol, NS, zflag, Edz, kmap, k_pad, nx_pad, nz_pad, pA, pBt, s);
}

// Tables of DenseEC over empty spaces (no instance has a dense z).
void Plan::empty_space(DenseSpace& d, hipStream_t s) {
  const int n = n_inst;
  const int64_t NYa = std::max<int64_t>(NY, 1);
  d.h_theta.assign(n, INT64_MAX);
  d.h_K.assign(n, 0);
  d.h_roww.assign(n, 0);
  d.h_hboff.assign(n, 0);
  d.d_theta = A.alloc<int64_t>(n, s);
  fill_i64(d.d_theta, n, INT64_MAX, s);
  d.d_hboff = A.alloc<int64_t>(n, s);
  fill_i64(d.d_hboff, n, 0, s);
  d.d_roww = A.alloc<int32_t>(n, s);
  fill_i32(d.d_roww, n, 0, s);
  d.d_cwmoff = A.alloc<int64_t>(n, s);
  fill_i64(d.d_cwmoff, n, 0, s);
  d.Ehot = A.alloc<int32_t>(NY + 1, s);
  fill_i32(d.Ehot, NY + 1, 0, s);
  d.hotrow = A.alloc<int32_t>(NYa, s);
  fill_i32(d.hotrow, NYa, -1, s);
  d.cptr = A.alloc<int32_t>(NY + 1, s);
  fill_i32(d.cptr, NY + 1, 0, s);
  d.NHb = 0;
  d.hb = A.alloc<uint32_t>(4, s);
  fill_u32(d.hb, 4, 0u, s);
  d.NCold = 0;
  d.ccol = A.alloc<int32_t>(1, s);
  fill_i32(d.ccol, 1, 0, s);
  d.wptr = A.alloc<int32_t>(1, s);
  fill_i32(d.wptr, 1, 0, s);
  d.rcode = A.alloc<int32_t>(std::max<int64_t>(NRp, 1), s);
  fill_i32(d.rcode, std::max<int64_t>(NRp, 1), -1, s);
}

// Tables of DenseEC over one z space: hot keys as bit rows over the space's
// local index, cold entries window-major, per-entry codes of R's CSR.
void Plan::build_space(DenseSpace& d, const int32_t* zmap, const int32_t* cnt_a, const int32_t* cnt_b,
                       const std::vector<int32_t>* hist_pre, Arena& T, hipStream_t s) {
  const int n = n_inst;
  const int64_t NSa = std::max<int64_t>(NS, 1), NYa = std::max<int64_t>(NY, 1);
  std::vector<int32_t> h_hist;
  if (hist_pre) {
    h_hist = *hist_pre;
  } else {
    int32_t* hist = T.alloc<int32_t>(int64_t(n) * 32, s);
    hot_histogram(cnt_a, cnt_b, dR, NY, y_base, n, hist, s);
    h_hist.resize(size_t(n) * 32);
    d2h(h_hist.data(), hist, size_t(n) * 32, s);
    if (d.h_base.empty()) {
      d.h_base.resize(n + 1);
      d2h(d.h_base.data(), d.base, n + 1, s);
    }
    sync(s);
  }

  // hot join keys: S row covering at least theta of the space
  const double hot_frac = env_double("JP_HOT_MIN_FRACTION", 1.0 / 128.0);
  d.h_theta.assign(n, INT64_MAX);
  d.h_K.assign(n, 0);
  d.h_roww.assign(n, 0);
  d.h_hboff.assign(n, 0);
  int64_t hb_words = 0;
  for (int i = 0; i < n; ++i) {
    int64_t zd = d.h_base[i + 1] - d.h_base[i];
    d.h_hboff[i] = hb_words;
    if (zd <= 0) continue;
    int64_t nwin = (zd + DW_BITS - 1) / DW_BITS;
    d.h_roww[i] = int32_t(nwin * DW_WORDS);
    int64_t th = std::max<int64_t>(2, int64_t(std::ceil(double(zd) * hot_frac)));
    int b = 0;
    while ((int64_t(1) << b) < th) ++b;
    // raise the bucket until at most kmax keys qualify
    auto count_from = [&](int bb) {
      int64_t c = 0;
      for (int q = bb; q < 32; ++q) c += h_hist[size_t(i) * 32 + q];
      return c;
    };
    const int kmax = opt.k_hot_max > 0 ? std::min(opt.k_hot_max, 1024)
                                        : (h_rec[i].valid && h_rec[i].k_hot_max > 0 ? h_rec[i].k_hot_max : 256);
    while (b < 31 && count_from(b) > kmax) ++b;
    int64_t K = count_from(b);
    d.h_theta[i] = int64_t(1) << b;
    d.h_K[i] = K;
    hb_words += K * d.h_roww[i];
  }
  d.d_theta = A.alloc<int64_t>(n, s);
  h2d(d.d_theta, d.h_theta.data(), n, s);
  d.d_hboff = A.alloc<int64_t>(n, s);
  h2d(d.d_hboff, d.h_hboff.data(), n, s);
  d.d_roww = A.alloc<int32_t>(n, s);
  h2d(d.d_roww, d.h_roww.data(), n, s);
  int32_t* hot = T.alloc<int32_t>(NYa, s);
  hot_flags(cnt_a, cnt_b, dR, NY, y_base, n, d.d_theta, hot, s);
  d.Ehot = A.alloc<int32_t>(NY + 1, s);
  scan_excl_i32(hot, d.Ehot, NY, s, T);
  d.hotrow = A.alloc<int32_t>(NYa, s);
  int64_t n_hot = 0;
  for (int i = 0; i < n; ++i) n_hot += d.h_K[i];
  int32_t* hotlist = T.alloc<int32_t>(std::max<int64_t>(n_hot, 1), s);
  hot_rank(hot, d.Ehot, NY, n_hot, y_base, n, dR, hotlist, d.hotrow, s);
  d.NHb = hb_words;
  d.hb = A.alloc<uint32_t>(std::max<int64_t>(hb_words, 4), s);
  fill_u32(d.hb, hb_words, 0u, s);
  build_hot_bits(hotlist, n_hot, sptr, scol, NS, d.hotrow, y_base, zmap, d.d_hboff, d.d_roww, n, d.hb, s, T);

  // cold entries: CSR by y over the space's local index (ascending in each row)
  int32_t* ccol_y = T.alloc<int32_t>(NSa, s);
  d.cptr = A.alloc<int32_t>(NY + 1, s);
  int32_t* d_ncold = T.alloc<int32_t>(1, s);
  int32_t* crow = T.alloc<int32_t>(NSa, s);  // row of each cold entry
  filter_rows(true, Ey, scol, NS, zmap, NZ, hot, ccol_y, crow, d.cptr, NY, d_ncold, s, T);
  int32_t ncold = 0;
  d2h(&ncold, d_ncold, 1, s);
  sync(s);
  d.NCold = ncold;

  // cold entries in window-major order with per-(window, key) segment bounds
  std::vector<int64_t> h_cwoff(n, 0), h_cwmoff(n, 0);
  int64_t cw_total = 0, cwm_total = 0;
  for (int i = 0; i < n; ++i) {
    h_cwoff[i] = cw_total;
    h_cwmoff[i] = cwm_total;
    int64_t zd = d.h_base[i + 1] - d.h_base[i];
    if (zd > 0) {
      int64_t ny = h_ybase[i + 1] - h_ybase[i], nwin = (zd + DW_BITS - 1) / DW_BITS;
      cw_total += ny * (nwin + 1);
      cwm_total += ny * nwin;
    }
  }
  if (cwm_total >= INT32_MAX) throw Error(JP_ENOMEM, "cold segment table too large");
  int64_t* d_offs = T.alloc<int64_t>(2 * int64_t(n), s);
  h2d(d_offs, h_cwoff.data(), n, s);
  d.d_cwmoff = A.alloc<int64_t>(n, s);
  h2d(d.d_cwmoff, h_cwmoff.data(), n, s);
  int32_t* cw = T.alloc<int32_t>(std::max<int64_t>(cw_total, 1), s);
  d.wptr = A.alloc<int32_t>(cwm_total + 1, s);
  d.ccol = A.alloc<int32_t>(std::max<int64_t>(d.NCold, 1), s);
  if (cw_total > 0) {
    cold_windows(d.cptr, ccol_y, crow, NY, d.NCold, y_base, d.base, n, d_offs, cw, s);
    cold_window_major(ccol_y, crow, NY, d.NCold, y_base, d.base, n, cw, d_offs, d.d_cwmoff, cwm_total, d.wptr, d.ccol,
                      s, T);
  } else {
    fill_i32(d.wptr, 1, 0, s);
  }
  d.rcode = A.alloc<int32_t>(std::max<int64_t>(NRp, 1), s);
  int32_t* ycode = T.alloc<int32_t>(NYa, s);
  row_codes(rcol, NRp, d.hotrow, d.cptr, NY, ycode, d.rcode, s);
}

// Pivot split of the DenseEC rows.  For an instance whose most shared hot key
// p (rank 0) lies in at least a quarter of its rows and covers at least half
// of its dense z, a row x holding p has
//   C[x] = S_dense[p]  disjoint-union  (OR over its other keys of S_dense[y] minus S_dense[p]),
// so its count is |S_dense[p]| plus a count over the dense z outside
// S_dense[p] (space 1), which is at most half as wide.  Rows without p keep
// space 0.  Exact for every row; only the count pass uses it.
// the automatic split needs rows of more than this many dense z (and enough cells)
constexpr int64_t PIVOT_MIN_DENSE_Z = 16384;

void Plan::pivot_split(Arena& T, hipStream_t s) {
  const int n = n_inst;
  n_piv = 0;
  // JP_PIVOT: 0 disables the split, 2 takes every rank-0 hot key as a pivot (tests)
  const double mode = env_double("JP_PIVOT", 1.0);
  if (mode == 0.0) return;
  DenseSpace& d0 = ds[0];
  // The split pays only for an instance with dense z beyond one window and
  // many (x, dense z) cells (its second set of tables costs plan time in
  // proportion to its tuples): candidates are decided from host-known sizes
  // before any device work.
  const double min_cells = env_double("JP_PIVOT_MIN_CELLS", 1e11);
  std::vector<char> cand(n, 0);
  bool any = false;
  for (int i = 0; i < n; ++i) {
    const int64_t nx = h_xbase[i + 1] - h_xbase[i], zd = h_zdbase[i + 1] - h_zdbase[i];
    cand[i] = d0.h_K[i] > 0 && (mode == 2.0 || (zd > PIVOT_MIN_DENSE_Z && double(nx) * double(zd) >= min_cells));
    any = any || cand[i];
  }
  if (!any) return;
  int32_t* info = T.alloc<int32_t>(3 * int64_t(n), s);
  d_piv = A.alloc<int32_t>(n, s);
  pivot_info(d0.hotrow, NY, y_base, n, dR, sptr, spptr, d_piv, info, s);
  std::vector<int32_t> h_info(3 * size_t(n));
  d2h(h_info.data(), info, 3 * size_t(n), s);
  sync(s);
  h_piv.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    const int32_t p = h_info[3 * i], dr = h_info[3 * i + 1], cnt = h_info[3 * i + 2];
    const int64_t nx = h_xbase[i + 1] - h_xbase[i], zd = h_zdbase[i + 1] - h_zdbase[i];
    if (p >= 0 && cand[i] && (mode == 2.0 || (4 * int64_t(dr) >= nx && 2 * int64_t(cnt) >= zd))) {
      h_piv[i] = p;
      ++n_piv;
    }
  }
  if (n_piv == 0) return;
  h2d(d_piv, h_piv.data(), n, s);
  const int64_t NZda = std::max<int64_t>(NZd, 1), NSa = std::max<int64_t>(NS, 1), NXa = std::max<int64_t>(NX, 1);
  int32_t* inP = T.alloc<int32_t>(NZda, s);
  fill_i32(inP, NZd, 0, s);
  mark_pivot(Ey, scol, NS, y_base, n, d_piv, zflag, Edz, inP, s);
  int32_t* rflag = T.alloc<int32_t>(NZda, s);
  resid_flags(inP, NZd, zd_base, n, d_piv, rflag, s);
  int32_t* Erd = T.alloc<int32_t>(NZd + 1, s);
  scan_excl_i32(rflag, Erd, NZd, s, T);
  DenseSpace& d1 = ds[1];
  d1.base = A.alloc<int32_t>(n + 1, s);
  gather_bases(Erd, zd_base, n, d1.base, s);
  int32_t* zmap1 = T.alloc<int32_t>(std::max<int64_t>(NZ, 1), s);
  zmap_resid(zflag, Edz, rflag, Erd, NZ, z_base, d1.base, n, zmap1, s);
  int32_t* f1 = T.alloc<int32_t>(NSa, s);
  space_flags(scol, NS, zmap1, f1, s);
  int32_t* E1 = T.alloc<int32_t>(NS + 1, s);
  scan_excl_i32(f1, E1, NS, s, T);
  int32_t* cnt1 = T.alloc<int32_t>(NY + 1, s);
  remap_rowptr(sptr, E1, NY, cnt1, s);
  build_space(d1, zmap1, cnt1, nullptr, nullptr, T, s);

  // rows holding their pivot, and the base count |S_dense[p]| = (dense z) - (space-1 z)
  int32_t* rf = T.alloc<int32_t>(NXa, s);
  row_pivot_flags(rptr, rcol, NX, x_base, n, d_piv, rf, s);
  int32_t* Er = T.alloc<int32_t>(NX + 1, s);
  scan_excl_i32(rf, Er, NX, s, T);
  int32_t np = 0;
  d2h(&np, Er + NX, 1, s);
  sync(s);
  NRowsP = np;
  NRowsN = NX - np;
  rows_p = A.alloc<int32_t>(std::max<int64_t>(NRowsP, 1), s);
  rows_n = A.alloc<int32_t>(std::max<int64_t>(NRowsN, 1), s);
  split_rows(rf, Er, NX, rows_p, rows_n, s);
  std::vector<int32_t> h_pc(n, 0);
  for (int i = 0; i < n; ++i)
    if (h_piv[i] >= 0) h_pc[i] = (h_zdbase[i + 1] - h_zdbase[i]) - (d1.h_base[i + 1] - d1.h_base[i]);
  d_pivcnt = A.alloc<int32_t>(n, s);
  h2d(d_pivcnt, h_pc.data(), n, s);
}

RowCtx Plan::ctx(int space) const {
  const DenseSpace& d = ds[space];
  RowCtx c;
  c.n_inst = n_inst;
  c.n_x = NX;
  c.max_z_range = 0;
  c.max_zd_range = 0;
  c.max_hot = 0;
  c.narrow = 0;
  c.by_width = space == 0 && nar_listed;
  for (int k = 0; k < N_WIDTH_CLASSES; ++k) {  // listed for space 0 only
    c.nar_x0[k] = c.by_width ? nar_x0[k] : nullptr;
    c.nar_base[k] = c.by_width ? nar_base[k] : nullptr;
    c.nar_m[k] = c.by_width ? nar_m[k] : 0;
    c.nar_rows[k] = c.by_width ? nar_rows[k] : 0;
    if (k < N_WIDTH_CLASSES - 1 && c.nar_m[k] > 0) c.narrow |= 1 << k;
  }
  for (int i = 0; i < n_inst; ++i) {
    c.max_z_range = std::max<int64_t>(c.max_z_range, h_zbase[i + 1] - h_zbase[i]);
    if (!d.h_base.empty()) c.max_zd_range = std::max<int64_t>(c.max_zd_range, d.h_base[i + 1] - d.h_base[i]);
    if (!d.h_K.empty()) c.max_hot = std::max<int64_t>(c.max_hot, d.h_K[i]);
  }
  c.x_base = x_base;
  c.z_base = z_base;
  c.zd_base = d.base;
  c.rptr = rptr;
  c.rcol = rcol;
  c.spptr = spptr;
  c.spcol = spcol;
  c.hotrow = d.hotrow;
  c.Ehot = d.Ehot;
  c.y_base = y_base;
  c.rcode = d.rcode;
  c.wptr = d.wptr;
  c.cwm_off = d.d_cwmoff;
  c.hb_off = d.d_hboff;
  c.row_words = d.d_roww;
  c.hb = d.hb;
  c.cptr = d.cptr;
  c.ccol = d.ccol;
  c.dz2z = dz2z;
  c.seg0 = seg0;
  c.seglen = seglen;
  c.wgroup = opt.window_group;
  if (c.wgroup == 0 && !h_rec.empty() && h_rec[0].valid) c.wgroup = h_rec[0].window_group;  // tuned
  c.light_max = light_max;
  c.med_max = med_max;
  return c;
}

// ---------------------------------------------------------------- execute
void Plan::execute(hipStream_t s) {
  stream = s;
  stream_used = true;
  const int64_t NXa = std::max<int64_t>(NX, 1);
  if (!w) {
    w = A.alloc<int64_t>(NXa, s);
    cnt_sp = A.alloc<int32_t>(NXa, s);
    cnt_de = A.alloc<int32_t>(NXa, s);
    cnt_all = A.alloc<int32_t>(NXa, s);
    off_all = A.alloc<int64_t>(NX + 1, s);
    off_de = A.alloc<int64_t>(NX + 1, s);
    off_sp = A.alloc<int64_t>(NX + 1, s);
    tot = A.alloc<int64_t>(3 * int64_t(n_inst), s);
    heavy_list = A.alloc<int32_t>(sparse_list_ints(NX), s);
    seg0 = A.alloc<int32_t>(std::max<int64_t>(NRp, 1), s);
    seglen = A.alloc<int32_t>(std::max<int64_t>(NRp, 1), s);
    XA.set_replay(true);
  }
  const bool graph = (opt.flags & JP_FLAG_GRAPH) != 0;
  const bool timing = (opt.flags & JP_FLAG_TIMING) != 0 && !graph;
  if (timing && !ev[0]) {
    for (auto& e : ev) JP_HIP(hipEventCreate(&e));
  }
  if (graph && graph_exec) {
    JP_HIP(hipGraphLaunch(graph_exec, s));
  } else if (graph && warm) {
    // Second run: every temporary is a replayed block, so the pass records
    // without allocating.  It is recorded on a private stream (the caller's may
    // be the null stream, which cannot capture) and launched on the caller's.
    if (!cap_stream) JP_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    JP_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      run_count_pass(cap_stream, false, false);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    JP_HIP(hipStreamEndCapture(cap_stream, &graph_));
    JP_HIP(hipGraphInstantiate(&graph_exec, graph_, nullptr, nullptr, 0));
    JP_HIP(hipGraphLaunch(graph_exec, s));
  } else {
    run_count_pass(s, timing, allow_aux && !timing && !graph);
  }
  warm = true;
  executed = true;
  offsets_ready = false;
  h_tot.clear();
}

void Plan::run_count_pass(hipStream_t s, bool timing, bool aux_ok) {
  XA.rewind();
  RowCtx c = ctx();
  if (timing) JP_HIP(hipEventRecord(ev[0], s));
  // The sparse and dense parts read the plan's tables and write disjoint
  // outputs; with work in both, the dense part runs on the auxiliary stream
  // (it allocates nothing from the pass's arena) so the two overlap.
  static const bool one_stream = env_double("JP_COUNT_ONE_STREAM", 0.0) != 0.0;  // for comparisons
  const bool split = aux_ok && !one_stream && NSp > 0 && NZd > 0;
  hipStream_t sd = s;
  if (split) {
    if (!aux_stream) {
      JP_HIP(hipStreamCreateWithFlags(&aux_stream, hipStreamNonBlocking));
      JP_HIP(hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming));
      JP_HIP(hipEventCreateWithFlags(&ev_join, hipEventDisableTiming));
    }
    JP_HIP(hipEventRecord(ev_fork, s));
    JP_HIP(hipStreamWaitEvent(aux_stream, ev_fork, 0));
    sd = aux_stream;
  }
  auto dense_part = [&](hipStream_t st) {
    if (NZd > 0 && use_mfma) {
      dense_mfma_count(pA, pBt, k_pad, NX, nx_pad, NZd, nz_pad, cnt_de, d_mfma_steps, mfma_tile, st);
    } else if (NZd > 0 && n_piv > 0) {
      fill_i32(cnt_de, NX, 0, st);
      dense_ec_rows(c, rows_n, NRowsN, nullptr, cnt_de, st);
      dense_ec_rows(ctx(1), rows_p, NRowsP, d_pivcnt, cnt_de, st);
    } else if (NZd > 0) {
      dense_ec(c, 0, NX, cnt_de, nullptr, nullptr, 0, st);
    } else {
      fill_i32(cnt_de, NX, 0, st);
    }
  };
  if (split) dense_part(sd);
  sparse_row_work(c, 0, NX, 0, NRp, w, seg0, seglen, s, XA);
  if (NSp > 0) sparse_bmm(c, 0, NX, w, cnt_sp, nullptr, nullptr, heavy_list, s);
  else fill_i32(cnt_sp, NX, 0, s);
  if (timing) JP_HIP(hipEventRecord(ev[1], s));
  if (!split) dense_part(s);
  if (split) {
    JP_HIP(hipEventRecord(ev_join, sd));
    JP_HIP(hipStreamWaitEvent(s, ev_join, 0));
  }
  if (timing) JP_HIP(hipEventRecord(ev[2], s));
  // per-instance totals now; the row offsets only when a list or the offsets are asked for (ensure_offsets)
  inst_sums(cnt_sp, cnt_de, x_base, n_inst, NX, tot, s);
  if (timing) JP_HIP(hipEventRecord(ev[3], s));
}

// Row offsets of the last count pass (prefix sums of the per-row counts of
// each part), computed at the first call that needs them.
void Plan::ensure_offsets(hipStream_t s) {
  if (offsets_ready) return;
  Arena T(&B);
  add_counts(cnt_sp, cnt_de, NX, cnt_all, s);
  scan_excl_i32_to_i64(cnt_all, off_all, NX, s, T);
  scan_excl_i32_to_i64(cnt_de, off_de, NX, s, T);
  scan_excl_i32_to_i64(cnt_sp, off_sp, NX, s, T);
  T.release(s);
  offsets_ready = true;
}

void Plan::timings(jp_timings* t, hipStream_t s) {
  if (!executed || !ev[0]) throw Error(JP_ESTATE, "timings need JP_FLAG_TIMING and a jp_execute");
  sync(s);
  std::memset(t, 0, sizeof(*t));
  JP_HIP(hipEventElapsedTime(&t->sparse_ms, ev[0], ev[1]));
  JP_HIP(hipEventElapsedTime(&t->dense_ms, ev[1], ev[2]));
  JP_HIP(hipEventElapsedTime(&t->execute_ms, ev[0], ev[3]));
  if (evp[0]) {
    JP_HIP(hipEventElapsedTime(&t->map_ms, evp[0], evp[1]));
    JP_HIP(hipEventElapsedTime(&t->partition_ms, evp[1], evp[2]));
  }
}

void Plan::work(jp_timings* t, hipStream_t s) {
  if (!executed) throw Error(JP_ESTATE, "work counters need a jp_execute");
  int64_t* d = A.alloc<int64_t>(4, s);
  if (n_piv > 0) {
    fill_i64(d, 4, 0, s);
    work_rows(ctx(0), rows_n, NRowsN, w, d, s);
    work_rows(ctx(1), rows_p, NRowsP, w, d, s);
  } else {
    work_stats(ctx(), 0, NX, w, d, s);
  }
  int64_t wk[4];
  d2h(wk, d, 4, s);
  sync(s);
  A.give_back(d, s);
  t->sparse_join_rows = wk[3];
  t->n_r_kept = NRp;
  t->n_x = NX;
  t->dense_hot_words = wk[0];
  t->dense_row_words = wk[1];
  t->dense_cold_entries = wk[2];
  t->dense_mfma_ops = use_mfma ? 2 * NX * K_panel * NZd : 0;
  if (use_mfma) {
    int64_t steps = 0;
    d2h(&steps, d_mfma_steps, 1, s);
    sync(s);
    t->dense_mfma_issued_ops = steps * mfma_step_ops(mfma_tile);
  }
  if (use_mfma) t->dense_hot_words = t->dense_row_words = t->dense_cold_entries = 0;
}

void Plan::fetch_totals(hipStream_t s) {
  if (!executed) throw Error(JP_ESTATE, "count before execute");
  if (h_tot.empty()) {
    h_tot.resize(3 * size_t(n_inst));
    d2h(h_tot.data(), tot, h_tot.size(), s);
    sync(s);
  }
}

// Write pairs [first, first + max) of instance i's sorted `part` result.
int64_t Plan::materialize(int inst, int part, int64_t first, int64_t maxp, int32_t* ox, int32_t* oz, hipStream_t s) {
  fetch_totals(s);
  const int64_t count = h_tot[3 * size_t(inst) + size_t(part)];
  if (first > count) throw Error(JP_ERANGE, "first beyond the number of pairs");
  const int64_t nw = std::min(maxp, count - first);
  if (nw <= 0) return 0;
  const int64_t xb = h_xbase[inst], xe = h_xbase[inst + 1];
  ensure_offsets(s);
  const int64_t* off = part == JP_PART_ALL ? off_all : (part == JP_PART_DENSE ? off_de : off_sp);
  int64_t base = 0;
  d2h(&base, off + xb, 1, s);
  sync(s);
  const int64_t g0 = base + first, g1 = g0 + nw;
  Arena T(&B);
  int64_t* rows = T.alloc<int64_t>(2, s);
  int64_t* info = T.alloc<int64_t>(6, s);
  find_rows(off, xb, xe, g0, g1, rows, s);
  hipLaunchKernelGGL(k_slice_info, dim3(1), dim3(64), 0, s, off_de, off_sp, rows, info);
  JP_LAUNCH_CHECK();
  int64_t h[6];
  d2h(h, info, 6, s);
  sync(s);
  const int64_t xl = h[0], xh = h[1];
  const int64_t nde = (part == JP_PART_SPARSE) ? 0 : h[3] - h[2];
  const int64_t nsp = (part == JP_PART_DENSE) ? 0 : h[5] - h[4];
  RowCtx c = ctx();
  int32_t* lde = T.alloc<int32_t>(std::max<int64_t>(nde, 1), s);
  int32_t* lsp = T.alloc<int32_t>(std::max<int64_t>(nsp, 1), s);
  if (nde > 0) dense_ec(c, xl, xh, nullptr, off_de, lde, nde, s);
  if (nsp > 0) sparse_bmm(c, xl, xh, w + xl, nullptr, off_sp, lsp, T.alloc<int32_t>(sparse_list_ints(xh - xl), s), s);
  if (part == JP_PART_ALL)
    merge_write_n(xl, xh, off_de, off_sp, off_all, lde, lsp, nde, nsp, vals_x, vals_z, g0, g1, ox, oz, s);
  else if (part == JP_PART_DENSE)
    merge_write_n(xl, xh, off_de, off_de, off_de, lde, nullptr, nde, 0, vals_x, vals_z, g0, g1, ox, oz, s);
  else
    merge_write_n(xl, xh, off_sp, off_sp, off_sp, lsp, nullptr, nsp, 0, vals_x, vals_z, g0, g1, ox, oz, s);
  sync(s);
  T.release(s);
  return nw;
}

void Plan::stats(int i, jp_stats* st) const {
  st->n_x = h_xbase[i + 1] - h_xbase[i];
  st->n_y = h_ybase[i + 1] - h_ybase[i];
  st->n_z = h_zbase[i + 1] - h_zbase[i];
  st->n_r_kept = h_rpbase[i + 1] - h_rpbase[i];
  st->out_j = h_outj[i];
  st->tau = h_tau[i];
  st->n_z_dense = h_zdbase[i + 1] - h_zdbase[i];
  st->k_hot = ds[0].h_K.empty() ? 0 : ds[0].h_K[i];
  st->footprint_bytes = n_inst == 1 ? A.bytes() : A.bytes() / n_inst;
  st->dense_mfma = use_mfma ? 1 : 0;
  st->peak_bytes = B.peak;
  st->map_direct = map_direct;
  st->strategy = JP_STRATEGY_HYBRID;
  st->pivot_cover = (n_piv > 0 && h_piv[i] >= 0) ? int64_t(h_zdbase[i + 1] - h_zdbase[i]) -
                                                       int64_t(ds[1].h_base[i + 1] - ds[1].h_base[i])
                                                 : 0;
}

}  // namespace jp

// ================================================================== C ABI

struct jp_batch {
  Plan p;
};

namespace {

jp_status check_cols(const int32_t* a, const int32_t* b, int64_t n, const char* what) {
  if (n < 0) return fail(JP_EINVAL, std::string(what) + ": negative tuple count");
  if (n > INT32_MAX) return fail(JP_EINVAL, std::string(what) + ": more than 2^31-1 tuples");
  if (n > 0 && (!a || !b)) return fail(JP_EINVAL, std::string(what) + ": null column with n > 0");
  return JP_OK;
}

jp_status check_opt(const jp_options* o) {
  if (!o) return JP_OK;
  if (o->tau_mode != JP_TAU_AUTO && o->tau_mode != JP_TAU_FIXED) return fail(JP_EINVAL, "bad tau_mode");
  if (o->dense_kernel < 0 || o->dense_kernel > 2) return fail(JP_EINVAL, "bad dense_kernel");
  if (o->k_hot_max < 0 || o->k_hot_max > 1024) return fail(JP_EINVAL, "k_hot_max must be in [0, 1024]");
  if (o->flags & ~(JP_FLAG_TIMING | JP_FLAG_GRAPH | JP_FLAG_DIRECT_IDS)) return fail(JP_EINVAL, "unknown flag bits");
  if (o->workspace_limit_bytes < 0) return fail(JP_EINVAL, "negative workspace limit");
  if (o->tau_mode == JP_TAU_FIXED && o->dense_threshold < -1) return fail(JP_EINVAL, "dense_threshold < -1");
  if (o->window_group < 0 || o->window_group > 64) return fail(JP_EINVAL, "window_group must be in [0, 64]");
  if (o->strategy < JP_STRATEGY_AUTO || o->strategy > JP_STRATEGY_CLASSICAL) return fail(JP_EINVAL, "bad strategy");
  if (o->sparse_light_max < 0 || o->sparse_light_max > 1024) return fail(JP_EINVAL, "sparse_light_max must be in [0, 1024]");
  if (o->sparse_med_max < 0 || o->sparse_med_max > 8192 ||
      (o->sparse_med_max > 0 && o->sparse_med_max < (o->sparse_light_max > 0 ? o->sparse_light_max : 1024)))
    return fail(JP_EINVAL, "sparse_med_max must be 0 or in [sparse_light_max, 8192]");
  if (o->mfma_tile < 0 || o->mfma_tile > 2) return fail(JP_EINVAL, "mfma_tile must be 0, 1 or 2");
  if (o->reserved != 0) return fail(JP_EINVAL, "reserved option field must be 0");
  return JP_OK;
}

}  // namespace

jp_status jp::check_options(const jp_options* o) { return check_opt(o); }

namespace {

// Device scratch of jp_count_static: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device
// copy: the device address comes from hipGetSymbolAddress (per device, in
// static_scratch()) and only that address is handed to kernels.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(JP_STATIC_SCRATCH_MIB) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_static_mu[MAX_DEVICES];  // one call at a time per device and process
void* g_static_ptr[MAX_DEVICES] = {};  // device address of scratch, per device (set under g_static_mu)

// Device address of this device's scratch (looked up once per device).
void* static_scratch(int dev) {
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    JP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw Error(JP_EHIP, "hipGetSymbolAddress returned a null address for the static scratch");
    g_static_ptr[dev] = p;
  }
  return g_static_ptr[dev];
}

}  // namespace

extern "C" {

const char* jp_last_error(void) { return g_last_error.c_str(); }

jp_status jp_count_static(const int32_t* r_x, const int32_t* r_y, int64_t n_r, const int32_t* s_z,
                          const int32_t* s_y, int64_t n_s, const jp_options* opt, hipStream_t stream,
                          int64_t* total, int64_t* dense, int64_t* sparse) {
  jp_status st;
  if ((st = check_cols(r_x, r_y, n_r, "R")) != JP_OK) return st;
  if ((st = check_cols(s_z, s_y, n_s, "S")) != JP_OK) return st;
  if (n_r + n_s > JP_STATIC_MAX_TUPLES)
    return fail(JP_EINVAL, "jp_count_static takes at most " + std::to_string(JP_STATIC_MAX_TUPLES) +
                               " tuples (n_r + n_s); use jp_plan_create for larger queries");
  if ((st = check_opt(opt)) != JP_OK) return st;
  if (opt && (opt->flags & (JP_FLAG_TIMING | JP_FLAG_GRAPH)))
    return fail(JP_EINVAL, "jp_count_static takes neither JP_FLAG_TIMING nor JP_FLAG_GRAPH");
  if (opt && opt->strategy == JP_STRATEGY_CLASSICAL)
    return fail(JP_EINVAL, "jp_count_static runs the hybrid path");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
    (void)hipGetLastError();
    return fail(JP_EHIP, "no usable current HIP device");
  }
  std::lock_guard<std::mutex> lock(g_static_mu[dev]);
  return guarded([&] {
    Region region;
    region.base = static_cast<char*>(static_scratch(dev));
    region.size = STATIC_SCRATCH_BYTES;
    RegionScope scope(&region);  // every arena below carves from the scratch
    Plan p;
    p.allow_aux = false;  // no stream or event creation on this path
    jp_instance in{r_x, r_y, s_z, s_y, n_r, n_s};
    try {
      p.build(&in, 1, opt, stream);
      p.execute(stream);
      p.fetch_totals(stream);  // syncs: the scratch is free again when this returns
    } catch (...) {
      (void)hipStreamSynchronize(stream);  // no work of this call may still use the scratch
      throw;
    }
    if (total) *total = p.h_tot[0];
    if (dense) *dense = p.h_tot[1];
    if (sparse) *sparse = p.h_tot[2];
  });
}

jp_status jp_plan_create(const int32_t* r_x, const int32_t* r_y, int64_t n_r, const int32_t* s_z, const int32_t* s_y,
                         int64_t n_s, const jp_options* opt, hipStream_t stream, jp_plan** out) {
  if (!out) return fail(JP_EINVAL, "out is null");
  *out = nullptr;
  jp_status st;
  if ((st = check_cols(r_x, r_y, n_r, "R")) != JP_OK) return st;
  if ((st = check_cols(s_z, s_y, n_s, "S")) != JP_OK) return st;
  if ((st = check_opt(opt)) != JP_OK) return st;
  const int strat = opt ? opt->strategy : JP_STRATEGY_AUTO;
  if (strat == JP_STRATEGY_CLASSICAL && (opt->flags & JP_FLAG_GRAPH))
    return fail(JP_EINVAL, "the classical path takes no JP_FLAG_GRAPH");
  jp_plan* p = new (std::nothrow) jp_plan();
  if (!p) return fail(JP_ENOMEM, "host allocation failed");
  jp_instance in{r_x, r_y, s_z, s_y, n_r, n_s};
  st = guarded([&] {
    // f1 (Sec. 2.6): the classical solution when its deduplication costs less
    // than the mapping; the hybrid build samples OUT_J at its first read-back
    // and stops there if the classical path wins
    bool classical = strat == JP_STRATEGY_CLASSICAL;
    if (!classical) {
      p->p.f1_probe = strat == JP_STRATEGY_AUTO &&
                      (!opt || (opt->tau_mode == JP_TAU_AUTO && opt->dense_kernel == JP_DENSE_AUTO &&
                                !(opt->flags & JP_FLAG_GRAPH)));
      p->p.build(&in, 1, opt, stream);
      if (p->p.take_classical) {
        (void)hipStreamSynchronize(stream);
        p->p.~Plan();  // a fresh hybrid plan object, holding nothing
        new (&p->p) Plan();
        classical = true;
      }
    }
    if (classical) {
      p->c.reset(new ClassicalPlan());
      p->c->arena_limit(opt ? opt->workspace_limit_bytes : 0);
      p->c->build(r_x, r_y, n_r, s_z, s_y, n_s, opt && (opt->flags & JP_FLAG_TIMING), stream);
      if (p->c->out_j > JP_CLASSICAL_MAX_OUT_J) {
        if (strat == JP_STRATEGY_CLASSICAL)
          throw Error(JP_EINVAL, "the classical path takes at most 2^30 join rows");
        p->c.reset();  // the estimate was too low: the hybrid path
        p->p.build(&in, 1, opt, stream);
      }
    }
  });
  if (st != JP_OK) {
    jp_plan_destroy(p);
    return st;
  }
  *out = p;
  return JP_OK;
}

jp_status jp_execute(jp_plan* p, hipStream_t stream) {
  if (!p) return fail(JP_EINVAL, "plan is null");
  if (p->c) return guarded([&] { p->c->execute(stream); });
  return guarded([&] { p->p.execute(stream); });
}

jp_status jp_count(jp_plan* p, int64_t* total, int64_t* dense, int64_t* sparse, hipStream_t stream) {
  if (!p) return fail(JP_EINVAL, "plan is null");
  if (p->c)
    return guarded([&] {
      p->c->fetch_total(stream);
      if (total) *total = p->c->total;
      if (dense) *dense = 0;
      if (sparse) *sparse = p->c->total;
    });
  return guarded([&] {
    p->p.fetch_totals(stream);
    if (total) *total = p->p.h_tot[0];
    if (dense) *dense = p->p.h_tot[1];
    if (sparse) *sparse = p->p.h_tot[2];
  });
}

jp_status jp_materialize(jp_plan* p, jp_part part, int64_t first, int64_t max_pairs, int32_t* out_x, int32_t* out_z,
                         int64_t* n_written, hipStream_t stream) {
  if (!p || !n_written) return fail(JP_EINVAL, "plan or n_written is null");
  if (part < JP_PART_ALL || part > JP_PART_SPARSE) return fail(JP_EINVAL, "bad part");
  if (first < 0 || max_pairs < 0) return fail(JP_EINVAL, "negative first or max_pairs");
  if (max_pairs > 0 && (!out_x || !out_z)) return fail(JP_EINVAL, "null output with max_pairs > 0");
  *n_written = 0;
  if (p->c) return guarded([&] { *n_written = p->c->materialize(int(part), first, max_pairs, out_x, out_z, stream); });
  return guarded([&] { *n_written = p->p.materialize(0, int(part), first, max_pairs, out_x, out_z, stream); });
}

jp_status jp_row_info(jp_plan* p, jp_part part, int32_t* x_values, int64_t* row_offsets, hipStream_t stream) {
  if (!p) return fail(JP_EINVAL, "plan is null");
  if (part < JP_PART_ALL || part > JP_PART_SPARSE) return fail(JP_EINVAL, "bad part");
  if (p->c) return guarded([&] { p->c->row_info(int(part), x_values, row_offsets, stream); });
  return guarded([&] {
    Plan& q = p->p;
    if (x_values) d2h(x_values, q.vals_x, size_t(q.NX), stream);
    if (row_offsets) {
      if (!q.executed) throw Error(JP_ESTATE, "row offsets before execute");
      q.ensure_offsets(stream);
      const int64_t* off = part == JP_PART_ALL ? q.off_all : (part == JP_PART_DENSE ? q.off_de : q.off_sp);
      d2h(row_offsets, off, size_t(q.NX) + 1, stream);
    }
    sync(stream);
  });
}

jp_status jp_dense_z(jp_plan* p, int32_t* z_values, hipStream_t stream) {
  if (!p) return fail(JP_EINVAL, "plan is null");
  if (p->c) return JP_OK;  // the classical path has no dense z
  return guarded([&] {
    Plan& q = p->p;
    if (q.NZd > 0 && z_values) {
      Arena T(&q.B);
      int32_t* tmp = T.alloc<int32_t>(q.NZd, stream);
      jp::gather_values(q.vals_z, q.dz2z, q.NZd, tmp, stream);
      d2h(z_values, tmp, size_t(q.NZd), stream);
      sync(stream);
      T.release(stream);
    }
  });
}

jp_status jp_plan_stats(const jp_plan* p, jp_stats* s) {
  if (!p || !s) return fail(JP_EINVAL, "null argument");
  if (p->c) p->c->stats(s);
  else p->p.stats(0, s);
  return JP_OK;
}

jp_status jp_plan_timings(jp_plan* p, jp_timings* t, hipStream_t stream) {
  if (!p || !t) return fail(JP_EINVAL, "null argument");
  if (p->c) return guarded([&] { p->c->timings(t, stream); });
  return guarded([&] { p->p.timings(t, stream); });
}

jp_status jp_plan_work(jp_plan* p, jp_timings* t, hipStream_t stream) {
  if (!p || !t) return fail(JP_EINVAL, "null argument");
  if (p->c)
    return guarded([&] {
      if (!p->c->executed) throw Error(JP_ESTATE, "work counters need a jp_execute");
      std::memset(t, 0, sizeof(*t));
    });
  return guarded([&] { p->p.work(t, stream); });
}

void jp_plan_destroy(jp_plan* p) {
  if (!p) return;
  if (p->p.stream_used) (void)hipStreamSynchronize(p->p.stream);
  if (p->c) (void)hipStreamSynchronize(p->c->stream);
  delete p;
}

jp_status jp_batch_create(const jp_instance* inst, int32_t n_inst, const jp_options* opt, hipStream_t stream,
                          jp_batch** out) {
  if (!out) return fail(JP_EINVAL, "out is null");
  *out = nullptr;
  if (n_inst <= 0 || !inst) return fail(JP_EINVAL, "need at least one instance");
  jp_status st;
  int64_t sr = 0, ss = 0;
  for (int i = 0; i < n_inst; ++i) {
    if ((st = check_cols(inst[i].r_x, inst[i].r_y, inst[i].n_r, "R")) != JP_OK) return st;
    if ((st = check_cols(inst[i].s_z, inst[i].s_y, inst[i].n_s, "S")) != JP_OK) return st;
    sr += inst[i].n_r;
    ss += inst[i].n_s;
  }
  if (sr > INT32_MAX || ss > INT32_MAX) return fail(JP_EINVAL, "batch holds more than 2^31-1 tuples per side");
  if ((st = check_opt(opt)) != JP_OK) return st;
  if (opt && opt->strategy == JP_STRATEGY_CLASSICAL)
    return fail(JP_EINVAL, "batches run the hybrid path (JP_STRATEGY_CLASSICAL is for single plans)");
  jp_batch* b = new (std::nothrow) jp_batch();
  if (!b) return fail(JP_ENOMEM, "host allocation failed");
  st = guarded([&] { b->p.build(inst, n_inst, opt, stream); });
  if (st != JP_OK) {
    jp_batch_destroy(b);
    return st;
  }
  *out = b;
  return JP_OK;
}

jp_status jp_batch_execute(jp_batch* b, hipStream_t stream) {
  if (!b) return fail(JP_EINVAL, "batch is null");
  return guarded([&] { b->p.execute(stream); });
}

jp_status jp_batch_counts(jp_batch* b, int64_t* totals, hipStream_t stream) {
  if (!b || !totals) return fail(JP_EINVAL, "null argument");
  return guarded([&] {
    b->p.fetch_totals(stream);
    for (int i = 0; i < b->p.n_inst; ++i) totals[i] = b->p.h_tot[3 * size_t(i)];
  });
}

jp_status jp_batch_materialize(jp_batch* b, int32_t inst, jp_part part, int64_t first, int64_t max_pairs,
                               int32_t* out_x, int32_t* out_z, int64_t* n_written, hipStream_t stream) {
  if (!b || !n_written) return fail(JP_EINVAL, "batch or n_written is null");
  if (inst < 0 || inst >= b->p.n_inst) return fail(JP_EINVAL, "instance index out of range");
  if (part < JP_PART_ALL || part > JP_PART_SPARSE) return fail(JP_EINVAL, "bad part");
  if (first < 0 || max_pairs < 0) return fail(JP_EINVAL, "negative first or max_pairs");
  if (max_pairs > 0 && (!out_x || !out_z)) return fail(JP_EINVAL, "null output with max_pairs > 0");
  *n_written = 0;
  return guarded([&] { *n_written = b->p.materialize(inst, int(part), first, max_pairs, out_x, out_z, stream); });
}

jp_status jp_batch_timings(jp_batch* b, jp_timings* t, hipStream_t stream) {
  if (!b || !t) return fail(JP_EINVAL, "null argument");
  return guarded([&] { b->p.timings(t, stream); });
}

jp_status jp_batch_work(jp_batch* b, jp_timings* t, hipStream_t stream) {
  if (!b || !t) return fail(JP_EINVAL, "null argument");
  return guarded([&] { b->p.work(t, stream); });
}

jp_status jp_batch_stats(const jp_batch* b, int32_t inst, jp_stats* s) {
  if (!b || !s) return fail(JP_EINVAL, "null argument");
  if (inst < 0 || inst >= b->p.n_inst) return fail(JP_EINVAL, "instance index out of range");
  b->p.stats(inst, s);
  return JP_OK;
}

jp_status jp_digest_pairs(const int32_t* x, const int32_t* z, int64_t n, uint64_t* digest, hipStream_t stream) {
  if (n < 0) return fail(JP_EINVAL, "negative pair count");
  if (!digest || (n > 0 && (!x || !z))) return fail(JP_EINVAL, "null argument");
  return guarded([&] { digest_pairs(x, z, n, digest, stream); });
}

void jp_batch_destroy(jp_batch* b) {
  if (!b) return;
  if (b->p.stream_used) (void)hipStreamSynchronize(b->p.stream);
  delete b;
}

}  // extern "C"
