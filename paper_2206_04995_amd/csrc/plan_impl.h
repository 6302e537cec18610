// Plan object behind jp_plan / jp_batch: device state of one or more
// Join-Project instances after mapping and partition, plus execute results.
#pragma once

#include <string>
#include <vector>

#include <memory>

#include "../../include/jp.h"
#include "classical.h"
#include "pool.h"
#include "stages.h"

namespace jp {

void gather_values(const int32_t* vals, const int32_t* idx, int64_t n, int32_t* out, hipStream_t s);
void set_last_error(const std::string& m);  // message returned by jp_last_error() on this thread

// The tables of DenseEC over one z space (see stages.h): space 0 holds every
// dense z; space 1 holds, per instance with a pivot key, the dense z outside
// the pivot's S row, and serves the rows that contain the pivot.
struct DenseSpace {
  std::vector<int32_t> h_base;  // [n_inst+1] prefix of the instances' space sizes
  std::vector<int64_t> h_theta, h_K, h_hboff;
  std::vector<int32_t> h_roww;
  int32_t* base = nullptr;      // device copy of h_base
  int64_t *d_theta = nullptr, *d_hboff = nullptr, *d_cwmoff = nullptr;
  int32_t *d_roww = nullptr, *Ehot = nullptr, *hotrow = nullptr, *cptr = nullptr, *ccol = nullptr;
  int32_t *wptr = nullptr, *rcode = nullptr;
  uint32_t* hb = nullptr;
  int64_t NHb = 0, NCold = 0;
};

// Choices jp_tune stored for one shape signature (valid = false: none).
struct TuneRec {
  bool valid = false;
  double ratio = 0.0;  // c_de / c_sp of the threshold
  int32_t dense_kernel = JP_DENSE_AUTO;
  int32_t k_hot_max = 0;
  int32_t window_group = 0;
  int32_t sparse_light_max = 0;
  int32_t sparse_med_max = 0;
  int32_t mfma_tile = 0;
};

struct Plan {
  Budget B;       // device bytes held at once by the arenas below and the stages' temporaries
  Arena A{&B};    // persistent state
  int n_inst = 0;
  jp_options opt{};
  hipStream_t stream = nullptr;
  bool stream_used = false;
  bool executed = false;

  int64_t NR = 0, NS = 0, NRp = 0, NX = 0, NY = 0, NZ = 0, NZd = 0, NSp = 0;
  int map_direct = 0;  // bit 0: z ids by the direct-range mapping, bit 1: x ids
  bool f1_probe = false;        // build(): sample OUT_J at the first read-back and stop if f1 prefers classical
  bool take_classical = false;  // build() stopped there
  // SparseBMM count class bounds and the INT8-MFMA tile in effect (options, else tuned, else defaults)
  int light_max = 1024, med_max = 8192, mfma_tile = 0;
  std::vector<int32_t> h_rbase, h_sbase, h_rpbase, h_xbase, h_ybase, h_zbase, h_zdbase;
  std::vector<int64_t> h_outj, h_tau, h_tot;
  std::vector<TuneRec> h_rec;  // per instance

  // inputs (concatenated over instances)
  const int32_t *rx = nullptr, *ry = nullptr, *sz = nullptr, *sy = nullptr;
  int32_t *d_rbase = nullptr, *d_sbase = nullptr, *d_rpbase = nullptr;
  int32_t* d_minmax = nullptr;  // a batch: per-instance min and max of z, y, x (6 rows of n), from the gather
  // a batch read in place: device table of the instances' column pointers
  // (R.x, R.y, S.z, S.y; n each), used by the mapping instead of rx, ry, sz, sy
  const int32_t* const* d_cols = nullptr;
  // mapping
  int32_t *vals_x = nullptr, *vals_y = nullptr, *vals_z = nullptr;
  int32_t *x_base = nullptr, *y_base = nullptr, *z_base = nullptr;
  int32_t *rptr = nullptr, *rcol = nullptr, *sptr = nullptr, *scol = nullptr, *Ey = nullptr, *zfirst = nullptr;
  int32_t *m_z = nullptr, *dR = nullptr, *dS = nullptr;
  int64_t* d_outj = nullptr;
  // partition
  int64_t* d_tau = nullptr;
  int32_t *zflag = nullptr, *Edz = nullptr, *dz2z = nullptr, *zd_base = nullptr;
  int32_t *spptr = nullptr, *spcol = nullptr;
  DenseSpace ds[2];
  // pivot split of the DenseEC rows (space 1 in use iff n_piv > 0)
  int n_piv = 0;
  std::vector<int32_t> h_piv;
  int32_t *d_piv = nullptr, *d_pivcnt = nullptr, *rows_p = nullptr, *rows_n = nullptr;
  int64_t NRowsP = 0, NRowsN = 0;
  // INT8-MFMA count of the dense part (single-instance plans with a dense panel)
  bool use_mfma = false;
  int8_t *pA = nullptr, *pBt = nullptr;
  int64_t* d_mfma_steps = nullptr;  // staged steps the product's workgroups ran (early checks stop them)
  int64_t K_panel = 0, k_pad = 0, nx_pad = 0, nz_pad = 0, dense_keys0 = 0;
  // rows of the instances by dense width (class 0: at most NARROW_SMALL dense
  // z, 1: NARROW_MID, 2: NARROW_MAX, 3: more): per class, the first x of each
  // such instance and the running row count
  int32_t* nar_x0[N_WIDTH_CLASSES] = {};
  int32_t* nar_base[N_WIDTH_CLASSES] = {};
  int nar_m[N_WIDTH_CLASSES] = {};
  int64_t nar_rows[N_WIDTH_CLASSES] = {};
  std::vector<int32_t> h_nar_x0[N_WIDTH_CLASSES], h_nar_base[N_WIDTH_CLASSES];  // host copies (upload sources)
  bool nar_listed = false;
  void narrow_segments(hipStream_t s);
  void choose_dense_kernel(Arena& T, hipStream_t s);
  void build_space(DenseSpace& d, const int32_t* zmap, const int32_t* cnt_a, const int32_t* cnt_b,
                   const std::vector<int32_t>* hist_pre, Arena& T, hipStream_t s);
  void empty_space(DenseSpace& d, hipStream_t s);
  void pivot_split(Arena& T, hipStream_t s);
  // execute
  int64_t* w = nullptr;
  int32_t *seg0 = nullptr, *seglen = nullptr;  // per R entry: sparse S row of its key
  int32_t *cnt_sp = nullptr, *cnt_de = nullptr, *cnt_all = nullptr;
  int64_t *off_all = nullptr, *off_de = nullptr, *off_sp = nullptr, *tot = nullptr;
  bool offsets_ready = false;  // off_* hold the last count pass's row offsets

  // JP_FLAG_TIMING: events around the execute kernels and work counters
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t evp[3] = {nullptr, nullptr, nullptr};  // start of the plan, after mapping, after partition
  int32_t* heavy_list = nullptr;
  void work(jp_timings* t, hipStream_t s);

  // temporaries of the count pass, replayed on every execute (see Arena)
  Arena XA{&B};
  bool warm = false;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // the dense part of a count pass runs on aux_stream beside the sparse part
  // (they share no data), forked from and joined back to the caller's stream
  // by events; off for captured, timed and static passes
  bool allow_aux = true;
  hipStream_t aux_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  void run_count_pass(hipStream_t s, bool timing, bool aux_ok);
  void ensure_offsets(hipStream_t s);  // row offsets of the last count pass, computed on first use

  ~Plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (aux_stream) (void)hipStreamDestroy(aux_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : evp)
      if (e) (void)hipEventDestroy(e);
    XA.release(stream);
    A.release(stream);
  }
  void timings(jp_timings* t, hipStream_t s);
  void arena_limit(int64_t lim) { B.limit = lim; }
  void build(const jp_instance* inst, int n, const jp_options* o, hipStream_t s);
  void map(hipStream_t s);
  void partition(hipStream_t s);
  RowCtx ctx(int space = 0) const;
  void execute(hipStream_t s);
  void fetch_totals(hipStream_t s);
  int64_t materialize(int inst, int part, int64_t first, int64_t maxp, int32_t* ox, int32_t* oz, hipStream_t s);
  void stats(int i, jp_stats* st) const;
};

// argument checks of jp_options shared by every entry point (JP_OK or JP_EINVAL with the message set)
jp_status check_options(const jp_options* o);

int64_t tau_from_cost(int64_t nx, int64_t nz, int64_t ns, int64_t out_j, double c_de_over_sp, double c_fix_over_sp);
// shape signature of one instance, and the cost ratio c_de / c_sp stored for it by jp_tune
uint64_t shape_signature(int64_t nx, int64_t nz, int64_t ns, int64_t out_j);
bool tuned_record(uint64_t sig, TuneRec* rec);

}  // namespace jp

// The C-ABI plan object: a hybrid plan, or the classical path when c is set.
struct jp_plan {
  jp::Plan p;
  std::unique_ptr<jp::ClassicalPlan> c;
};
