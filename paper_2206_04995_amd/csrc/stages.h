// Launchers of the Join-Project stages (mapping, partition, SparseBMM,
// DenseEC, output).  All ids are global across the instances of a plan: the
// ids of instance i occupy [base[i], base[i+1]) of their id space.
#pragma once

#include "pool.h"

namespace jp {

// Window of the dense-z bitmaps, in bits (DenseEC processes one window of a
// row at a time).
constexpr int DW_BITS = 32768;
constexpr int DW_WORDS = DW_BITS / 32;
// count mode: rows of instances with at most this many dense z are counted
// with a quarter wave (NARROW_SMALL), a whole wave with one word per lane
// (NARROW_MID) or four words per lane (NARROW_MAX) per row
constexpr int NARROW_SMALL = 512;
constexpr int NARROW_MID = 2048;
constexpr int NARROW_MAX = 8192;
constexpr int N_WIDTH_CLASSES = 4;  // the three narrow classes and the window kernel's
// hot keys whose window slices a DenseEC workgroup stages in LDS
constexpr int T_STAGE = 3;

// ------------------------------------------------------------ mapping
// a batch's columns, one device pointer per instance (src[i], base[i + 1] -
// base[i] values), into one buffer dst (or nowhere, if dst is null); with
// mn/mx non-null also each instance's minimum and maximum (atomically merged
// into mn/mx, which fill_minmax prepares: 6 rows of n_inst, minima at rows 0, 2, 4)
void fill_minmax(int32_t* mm, int n_inst, hipStream_t s);
void gather_cols(const int32_t* const* src, const int32_t* base, int n_inst, int64_t n, int32_t* dst, int32_t* mn,
                 int32_t* mx, hipStream_t s);
// keys[i] = koff[inst(i)] + (v[i] - mn[inst(i)]); if payload is non-null,
// payload[i] = pay_src[i] (a column carried through the sort) or i
void make_keys(const int32_t* v, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff,
               const int32_t* mn, uint32_t* keys, uint32_t* payload, const int32_t* pay_src, hipStream_t s);
// A column carried through a sort by run keys: with it, run_ids writes the id of
// each sorted position (payload) and the key of the carried value under the
// layout (koff, mn) of the next sort (keys), instead of E.
struct RunCarry {
  const int32_t* v;
  const int64_t* koff;
  const int32_t* mn;
  uint32_t* keys;
  uint32_t* payload;
};
// ids of the runs of equal sorted keys: for each run id, first[id] = its first
// position and vals[id] = the original value of its key; first[runs] = n, and
// *total = runs if total is non-null.  If E is non-null, E[p] = runs started
// before position p (E[n] = runs); with carry, E is not written.  With table,
// table[key] = id for the key of every run (the entries of other keys are
// left as they are).
void run_ids(const uint32_t* keys, int64_t n, const int64_t* koff, const int32_t* mn, int n_inst, int32_t* E,
             int32_t* first, int32_t* vals, hipStream_t s, Arena& a, int32_t* total = nullptr,
             const RunCarry* carry = nullptr, int32_t* table = nullptr);
// out[i] = runs started before ebase[i] (i in [0, n_inst]), from first[] and the run count
void ids_at_bases(const int32_t* first, const int32_t* total, const int32_t* ebase, int n_inst, int32_t* out,
                  hipStream_t s);
// out[i] = E[ebase[i]] for i in [0, n_inst]
void gather_bases(const int32_t* E, const int32_t* ebase, int n_inst, int32_t* out, hipStream_t s);
// semi-join of R on S.y: keep[g] = 1 and yid[g] = id iff ry[g] occurs among the y values of its instance
void semijoin(const int32_t* ry, int64_t n, const int32_t* ebase, int n_inst, const int32_t* vals_y,
              const int32_t* y_base, int32_t* keep, int32_t* yid, hipStream_t s);
// same result through a direct-address table over the key space of S.y
// (table has key_space entries; ykeys are the y-sorted S keys, first[] their
// run starts and *total the run count)
void semijoin_direct(const int32_t* ry, int64_t n, const int32_t* ebase, int n_inst, const uint32_t* ykeys, int64_t ns,
                     const int32_t* first, const int32_t* total, const int64_t* koff, int64_t key_space,
                     const int32_t* mn, int32_t* table, int32_t* keep, int32_t* yid, hipStream_t s);
// Inputs of the fused semi-join of R: R's columns and instance bases, the y
// lookup (table over the S.y key space when table is non-null, else binary
// search in vals_y within y_base), and the layout of the x keys.
struct SemiJoinIn {
  const int32_t* rx;
  const int32_t* ry;
  // or, if non-null, one buffer per instance: element i of instance k is cx[k][i - ebase[k]]
  const int32_t* const* cx;
  const int32_t* const* cy;
  int64_t n;
  const int32_t* ebase;
  int n_inst;
  const int64_t* koff_y;
  const int32_t* ymin;
  const int32_t* table;
  const int32_t* vals_y;
  const int32_t* y_base;
  const int64_t* koff_x;
  const int32_t* xmin;
};
// semi-join of R on S.y with the kept tuples compacted in order: xk = their x
// keys, oy = their y ids, rpbase[i] = kept tuples before instance i (i in
// [0, n_inst]), *total = kept tuples
void semijoin_compact(const SemiJoinIn& in, uint32_t* xk, uint32_t* oy, int32_t* rpbase, int32_t* total,
                      hipStream_t s, Arena& a);
// Direct-range mapping (key space = the instances' stacked value ranges):
// h[key(v[i])] += 1 for every i with filter[i] >= 0 (filter may be null)
void key_hist(const int32_t* v, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff, const int32_t* mn,
              const int32_t* filter, int32_t* h, hipStream_t s);
// pres[k] = cnt[k] > 0
void presence(const int32_t* cnt, int64_t n_keys, int32_t* pres, hipStream_t s);
// for each present key k (cnt[k] > 0): id E[k], vals[id] = its value, m[id] = cnt[k] and
// first[id] = C[k] (m, first nullable); first[E[n_keys]] = C[n_keys]
void key_ids(const int32_t* cnt, int64_t n_keys, const int32_t* E, const int32_t* C, const int64_t* koff,
             const int32_t* mn, int n_inst, int32_t* vals, int32_t* m, int32_t* first, hipStream_t s);
// out[i] = E[koff[i]] for i in [0, n_inst]
void bases_from_koff(const int32_t* E, const int64_t* koff, int n_inst, int32_t* out, hipStream_t s);
// S into z order: position cur[zkey]++ gets the tuple's y key and z id Ez[zkey]
void scatter_z(const int32_t* sz, const int32_t* sy, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff_z,
               const int32_t* zmin, const int64_t* koff_y, const int32_t* ymin, const int32_t* Ez, int32_t* cur,
               uint32_t* yk, uint32_t* zid, hipStream_t s);
// kept R tuples (yid >= 0) grouped by x: rcol[cur[xkey]++] = yid
void scatter_x(const int32_t* rx, const int32_t* yid, int64_t n, const int32_t* ebase, int n_inst, const int64_t* koff_x,
               const int32_t* xmin, int32_t* cur, int32_t* rcol, hipStream_t s);
// m[i] = first[i + 1] - first[i]
void run_lengths(const int32_t* first, int64_t n_id, int32_t* m, hipStream_t s);
// h[v[i]] += 1; nbins > 0 (the key space, when known) picks direct LDS bins for a small space
void histogram(const uint32_t* v, int64_t n, int32_t* h, hipStream_t s, int64_t nbins = 0);
// out_j[inst] += sum over y of dR[y] * dS[y]
void out_j_per_inst(const int32_t* dR, const int32_t* dS, int64_t n_y, const int32_t* y_base, int n_inst,
                    int64_t* out_j, hipStream_t s);

// ---------------------------------------------------------- partition
// flag[z] = m_z[z] > tau[inst(z)]
void dense_flags(const int32_t* m_z, int64_t n_z, const int32_t* z_base, int n_inst, const int64_t* tau,
                 int32_t* flag, hipStream_t s);
// dz2z[Edz[z]] = z for dense z
void dense_index(const int32_t* flag, const int32_t* Edz, int64_t n_z, int32_t* dz2z, hipStream_t s);
// S entries filtered into a CSR over the rows of S in one pass: the entries
// whose z is sparse (cold = false: zsel = zflag, out = z), or the cold
// entries of a space (cold = true: zsel = zmap, hot = hot rows, out = local
// index); zsel has n_z entries; rowptr gets n_rows + 1 entries, *total the kept count;
// out_row (if not null) gets the row of each kept entry
void filter_rows(bool cold, const int32_t* Ey, const int32_t* scol, int64_t n, const int32_t* zsel, int64_t n_z,
                 const int32_t* hot, int32_t* out, int32_t* out_row, int32_t* rowptr, int64_t n_rows, int32_t* total,
                 hipStream_t s, Arena& a);
// rowptr_out[y] = E[rowptr[y]] for y in [0, n_y]
void remap_rowptr(const int32_t* rowptr, const int32_t* E, int64_t n_y, int32_t* out, hipStream_t s);
// The tables of DenseEC are built over a "space" of z: a map zmap[z] = local
// index of z in its instance's part of the space, or -1 if z is not in it.
// The count of key y in the space is cnt_a[y+1] - cnt_a[y] - (cnt_b ? cnt_b[y+1] - cnt_b[y] : 0).
//
// per-instance histogram of floor(log2(count in the space)) over y with dR > 0 (32 buckets)
void hot_histogram(const int32_t* cnt_a, const int32_t* cnt_b, const int32_t* dR, int64_t n_y, const int32_t* y_base,
                   int n_inst, int32_t* hist, hipStream_t s);
// hot[y] = 1 iff dR[y] > 0 and the count of y in the space >= theta[inst(y)]
void hot_flags(const int32_t* cnt_a, const int32_t* cnt_b, const int32_t* dR, int64_t n_y, const int32_t* y_base,
               int n_inst, const int64_t* theta, int32_t* hot, hipStream_t s);
// hot row bit sets over the space's local index (one lane per entry of a hot row;
// hotlist holds the n_hot hot keys, sptr is the CSR of S by y)
void build_hot_bits(const int32_t* hotlist, int64_t n_hot, const int32_t* sptr, const int32_t* scol, int64_t n_s,
                    const int32_t* hotrow, const int32_t* y_base, const int32_t* zmap, const int64_t* hb_off,
                    const int32_t* row_words, int n_inst, uint32_t* hb, hipStream_t s, Arena& a);
// per S entry: in the space
void space_flags(const int32_t* scol, int64_t n, const int32_t* zmap, int32_t* flag, hipStream_t s);
// space 0: all dense z
void zmap_dense(const int32_t* zflag, const int32_t* Edz, int64_t n_z, const int32_t* z_base, const int32_t* zd_base,
                int n_inst, int32_t* zmap, hipStream_t s);
// space 1: the dense z with rflag[dense index] set (Erd: exclusive scan of rflag)
void zmap_resid(const int32_t* zflag, const int32_t* Edz, const int32_t* rflag, const int32_t* Erd, int64_t n_z,
                const int32_t* z_base, const int32_t* zc_base, int n_inst, int32_t* zmap, hipStream_t s);
// piv[i] = hot key of rank 0 of instance i (or -1); info[3i..] = (piv, dR(piv), count of piv in the space)
void pivot_info(const int32_t* hotrow, int64_t n_y, const int32_t* y_base, int n_inst, const int32_t* dR,
                const int32_t* cnt_a, const int32_t* cnt_b, int32_t* piv, int32_t* info, hipStream_t s);
// inP[Edz[z]] = 1 for the dense z of each instance's pivot row
void mark_pivot(const int32_t* Ey, const int32_t* scol, int64_t n, const int32_t* y_base, int n_inst,
                const int32_t* piv, const int32_t* zflag, const int32_t* Edz, int32_t* inP, hipStream_t s);
// rflag[d] = 1 iff dense index d is of an instance with a pivot (piv >= 0) and not in its pivot row
void resid_flags(const int32_t* inP, int64_t n, const int32_t* zd_base, int n_inst, const int32_t* piv, int32_t* out,
                 hipStream_t s);
// flag[x] = 1 iff R row x holds the pivot of its instance
void row_pivot_flags(const int32_t* rptr, const int32_t* rcol, int64_t n_x, const int32_t* x_base, int n_inst,
                     const int32_t* piv, int32_t* flag, hipStream_t s);
// flagged rows to rows_p, the others to rows_n (E = exclusive scan of flag)
void split_rows(const int32_t* flag, const int32_t* E, int64_t n, int32_t* rows_p, int32_t* rows_n, hipStream_t s);

// ----------------------------------------------------------- row work
struct RowCtx {
  int n_inst;
  int64_t n_x;             // rows of all instances
  int64_t max_z_range;     // largest number of z ids of one instance
  int64_t max_zd_range;    // largest number of dense z ids of one instance
  int64_t max_hot;         // largest number of hot keys of one instance
  const int32_t* x_base;   // [n_inst+1]
  const int32_t* z_base;   // [n_inst+1]
  const int32_t* zd_base;  // [n_inst+1]
  const int32_t* rptr;     // [n_x+1]
  const int32_t* rcol;     // y ids
  // sparse part
  const int32_t* spptr;    // [n_y+1]
  const int32_t* spcol;    // z ids, ascending within a row
  // dense part
  const int32_t* hotrow;   // [n_y]: global hot row index or -1
  const int32_t* Ehot;     // [n_y+1] exclusive scan of hot flags
  const int32_t* y_base;   // [n_inst+1]
  const int64_t* hb_off;   // [n_inst] word offset of the instance's hot rows
  const int32_t* row_words;// [n_inst] words per hot row (multiple of DW_WORDS)
  const uint32_t* hb;      // hot rows
  const int32_t* cptr;     // [n_y+1] number of cold entries per y (cptr[y+1] - cptr[y])
  const int32_t* ccol;     // cold entries (local dense index), window-major: by window, then y, then z
  const int32_t* dz2z;     // [n_z_dense] dense index -> z id
  const int32_t* rcode;    // [n_r_kept] per R CSR entry: hot rank (>= 0), -2 - y (cold y), -1 (no dense entry)
  const int32_t* wptr;     // segment of (window w, y): ccol[wptr[k], wptr[k+1]), k = cwm_off[i] + w*Y_i + y - y_base[i]
  const int64_t* cwm_off;  // [n_inst] offset of the instance's segment table
  int wgroup;              // windows per workgroup of the count kernel (0: from dense_window_group)
  // rows by the dense width of their instance, class 0: 0 < dense z <= NARROW_SMALL,
  // 1: up to NARROW_MID, 2: up to NARROW_MAX, 3: more (space 0 only; set when the
  // partition listed them)
  int narrow;                  // bit k: class k has rows (k = 0, 1, 2)
  bool by_width;               // the classes are listed
  const int32_t* nar_x0[N_WIDTH_CLASSES];    // per class: first x of each instance of the class
  const int32_t* nar_base[N_WIDTH_CLASSES];  // per class: running count of their rows [nar_m + 1]
  int nar_m[N_WIDTH_CLASSES];
  int64_t nar_rows[N_WIDTH_CLASSES];
  // per R CSR entry j (filled by sparse_row_work): the sparse S row of its key
  const int32_t* seg0;     // first entry in spcol
  const int32_t* seglen;   // number of entries
  // SparseBMM count: rows with work <= light_max run one per wavefront, up to med_max one per workgroup
  int light_max;
  int med_max;
};

// hot rank of each hot y within its instance, by decreasing d_R (rows sharing it)
void hot_rank(const int32_t* hot, const int32_t* Ehot, int64_t n_y, int64_t n_hot, const int32_t* y_base, int n_inst,
              const int32_t* dR, int32_t* hotlist, int32_t* hotrow, hipStream_t s);
// per R CSR entry code (see RowCtx::rcode)
void row_codes(const int32_t* rcol, int64_t n, const int32_t* hotrow, const int32_t* cptr, int64_t n_y,
               int32_t* ycode, int32_t* rcode, hipStream_t s);
// cold segment table: cw[cw_off[i] + w * Y_i + (y - y_base[i])] = first cold entry of y with local dense
// index >= w * DW_BITS, for w in [0, nwin_i]; crow[p] = row of cold entry p
void cold_windows(const int32_t* cptr, const int32_t* ccol, const int32_t* crow, int64_t n_y, int64_t n_cold,
                  const int32_t* y_base, const int32_t* zd_base, int n_inst, const int64_t* cw_off, int32_t* cw,
                  hipStream_t s);
// Window-major copy of the cold entries: the entries of (window w, key y) of
// instance i are ccol_w[wptr[k], wptr[k + 1]) with k = cwm_off[i] + w * Y_i + (y - y_base[i]);
// wptr has cwm_total + 1 entries.
void cold_window_major(const int32_t* ccol, const int32_t* crow, int64_t n_y, int64_t n_cold, const int32_t* y_base,
                       const int32_t* zd_base, int n_inst, const int32_t* cw, const int64_t* cw_off,
                       const int64_t* cwm_off, int64_t cwm_total, int32_t* wptr, int32_t* ccol_w, hipStream_t s,
                       Arena& a);

// per-row work of the sparse part: w[x] = sum over y in R[x] of |S_sparse[y]|,
// for rows [x_lo, x_hi) whose CSR entries are [j_lo, j_hi)
void sparse_row_work(const RowCtx& c, int64_t x_lo, int64_t x_hi, int64_t j_lo, int64_t j_hi, int64_t* w,
                     int32_t* seg0, int32_t* seglen, hipStream_t s, Arena& a);
// SparseBMM count (cnt != null) or write (out != null, offsets relative to off[x_lo]);
// lists is scratch of sparse_list_ints(x_hi - x_lo) ints (the rows sorted by work)
int64_t sparse_list_ints(int64_t n_rows);
void sparse_bmm(const RowCtx& c, int64_t x_lo, int64_t x_hi, const int64_t* w, int32_t* cnt,
                const int64_t* off, int32_t* out, int32_t* lists, hipStream_t s);
// DenseEC count or write, bit-packed hot rows
// (write mode: out holds out_n values; writes past it are dropped)
void dense_ec(const RowCtx& c, int64_t x_lo, int64_t x_hi, int32_t* cnt, const int64_t* off, int32_t* out,
              int64_t out_n, hipStream_t s);
// DenseEC count over a list of rows, adding to cnt (zeroed by the caller);
// every row's count starts at base_cnt[instance] when base_cnt is given
void dense_ec_rows(const RowCtx& c, const int32_t* rows, int64_t n_rows, const int32_t* base_cnt, int32_t* cnt,
                   hipStream_t s);
// INT8-MFMA DenseEC for one instance with a dense panel: kmap[y] = panel key of y
// (a dense S entry and an R row; else -1), returns the number of panel keys (syncs s); panels A [nx_pad][k_pad]
// and Bt [nz_pad][k_pad] of 0/1 bytes; count pass writes cnt[0, nx)
int64_t panel_key_count(const int32_t* sptr, const int32_t* spptr, const int32_t* dR, int64_t n_y, int32_t* kmap,
                        Arena& T, hipStream_t s);
void build_panels(const int32_t* rptr, const int32_t* rcol, int64_t n_x, const int32_t* Ey, const int32_t* scol,
                  int64_t n_s, const int32_t* zflag, const int32_t* Edz, const int32_t* kmap, int64_t k_pad,
                  int64_t nx_pad, int64_t nz_pad, int8_t* A, int8_t* Bt, hipStream_t s);
// panel rows (x) and columns (dense z) padded to the product's tiles
int64_t mfma_pad_rows(int64_t n);
int64_t mfma_pad_cols(int64_t n);
int64_t mfma_pad_keys(int64_t n);
void dense_mfma_count(const int8_t* A, const int8_t* Bt, int64_t k_pad, int64_t nx, int64_t nx_pad, int64_t nz,
                      int64_t nz_pad, int32_t* cnt, int64_t* steps, int tile, hipStream_t s);
// int8 ops one workgroup of the given tile issues per staged step (2 * tile rows * tile columns * keys)
int64_t mfma_step_ops(int tile);
// windows per workgroup of the DenseEC count kernel (JP_DENSE_WINDOW_GROUP overrides)
int dense_window_group(int64_t max_hot, int nwin);

// algorithmic work of the count kernels over rows [x_lo, x_hi) (see jp_timings)
void work_stats(const RowCtx& c, int64_t x_lo, int64_t x_hi, const int64_t* w, int64_t* out4, hipStream_t s);
// the same sums over a list of rows, added to out4 (w indexed by x; nullable)
void work_rows(const RowCtx& c, const int32_t* rows, int64_t n_rows, const int64_t* w, int64_t* out4, hipStream_t s);

// ------------------------------------------------------------- output
// *acc (device) += sum over the n pairs of SplitMix64(key(x, z)), wrapping:
// the order-independent digest of a pair list
void digest_pairs(const int32_t* x, const int32_t* z, int64_t n, uint64_t* acc, hipStream_t s);
void add_counts(const int32_t* a, const int32_t* b, int64_t n, int32_t* out, hipStream_t s);
// tot[3i + {0, 1, 2}] = all, dense, sparse pairs of instance i, summed from the per-row counts
void inst_sums(const int32_t* cnt_sp, const int32_t* cnt_de, const int32_t* x_base, int n_inst, int64_t n_x,
               int64_t* tot, hipStream_t s);
// rows [lo, hi) covering global pair range [g0, g1) of an offset array
void find_rows(const int64_t* off, int64_t x_begin, int64_t x_end, int64_t g0, int64_t g1, int64_t* out2,
               hipStream_t s);
// Merge per-row sorted z lists: la (na entries, row offsets off_a) and lb
// (nb entries, offsets off_b; null for none) over rows [x_lo, x_hi); the pair
// of global rank g = off_out[x] + rank-in-row is written to out[g - g0] when
// g0 <= g < g1, as original values.
void merge_write_n(int64_t x_lo, int64_t x_hi, const int64_t* off_a, const int64_t* off_b, const int64_t* off_out,
                   const int32_t* la, const int32_t* lb, int64_t na, int64_t nb, const int32_t* vals_x,
                   const int32_t* vals_z, int64_t g0, int64_t g1, int32_t* out_x, int32_t* out_z, hipStream_t s);

}  // namespace jp
