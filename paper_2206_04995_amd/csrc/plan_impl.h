// Plan object behind jp_plan / jp_batch: device state of one or more
// Join-Project instances after mapping and partition, plus execute results.
#pragma once

#include <string>
#include <vector>

#include "../../include/jp.h"
#include "pool.h"
#include "stages.h"

namespace jp {

void gather_values(const int32_t* vals, const int32_t* idx, int64_t n, int32_t* out, hipStream_t s);
void set_last_error(const std::string& m);  // message returned by jp_last_error() on this thread

struct Plan {
  Arena A;
  int n_inst = 0;
  jp_options opt{};
  hipStream_t stream = nullptr;
  bool stream_used = false;
  bool executed = false;

  int64_t NR = 0, NS = 0, NRp = 0, NX = 0, NY = 0, NZ = 0, NZd = 0, NSp = 0, NCold = 0, NHb = 0;
  std::vector<int32_t> h_rbase, h_sbase, h_rpbase, h_xbase, h_ybase, h_zbase, h_zdbase;
  std::vector<int64_t> h_outj, h_tau, h_theta, h_K, h_hboff, h_tot;
  std::vector<int32_t> h_roww;

  // inputs (concatenated over instances)
  const int32_t *rx = nullptr, *ry = nullptr, *sz = nullptr, *sy = nullptr;
  int32_t *d_rbase = nullptr, *d_sbase = nullptr, *d_rpbase = nullptr;
  // mapping
  int32_t *vals_x = nullptr, *vals_y = nullptr, *vals_z = nullptr;
  int32_t *x_base = nullptr, *y_base = nullptr, *z_base = nullptr;
  int32_t *rptr = nullptr, *rcol = nullptr, *sptr = nullptr, *scol = nullptr, *Ey = nullptr, *zfirst = nullptr;
  int32_t *m_z = nullptr, *dR = nullptr, *dS = nullptr;
  int64_t* d_outj = nullptr;
  // partition
  int64_t *d_tau = nullptr, *d_theta = nullptr, *d_hboff = nullptr;
  int32_t *d_roww = nullptr, *zflag = nullptr, *Edz = nullptr, *dz2z = nullptr, *zd_base = nullptr;
  int32_t *spptr = nullptr, *spcol = nullptr, *Ehot = nullptr, *hotrow = nullptr, *cptr = nullptr, *ccol = nullptr;
  uint32_t* hb = nullptr;
  int32_t *rcode = nullptr, *wptr = nullptr;
  int64_t* d_cwmoff = nullptr;
  // execute
  int64_t* w = nullptr;
  int32_t *cnt_sp = nullptr, *cnt_de = nullptr, *cnt_all = nullptr;
  int64_t *off_all = nullptr, *off_de = nullptr, *off_sp = nullptr, *tot = nullptr;

  // JP_FLAG_TIMING: events around the execute kernels and work counters
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  int32_t* heavy_list = nullptr;
  void work(jp_timings* t, hipStream_t s);

  // temporaries of the count pass, replayed on every execute (see Arena)
  Arena XA;
  bool warm = false;
  hipGraph_t graph_ = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  void run_count_pass(hipStream_t s, bool timing);

  ~Plan() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
    XA.release(stream);
    A.release(stream);
  }
  void timings(jp_timings* t, hipStream_t s);
  void arena_limit(int64_t lim) {
    A.set_limit(lim);
    XA.set_limit(lim);
  }
  void build(const jp_instance* inst, int n, const jp_options* o, hipStream_t s);
  void map(hipStream_t s);
  void partition(hipStream_t s);
  RowCtx ctx() const;
  void execute(hipStream_t s);
  void fetch_totals(hipStream_t s);
  int64_t materialize(int inst, int part, int64_t first, int64_t maxp, int32_t* ox, int32_t* oz, hipStream_t s);
  void stats(int i, jp_stats* st) const;
};

int64_t tau_from_cost(int64_t nx, int64_t nz, int64_t ns, int64_t out_j, double c_de_over_sp, double c_fix_over_sp);

}  // namespace jp
