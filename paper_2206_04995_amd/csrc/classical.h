// The classical Join-Project path (hash join + device hash-set deduplication)
// and the strategy choice f1; see classical.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/jp.h"
#include "pool.h"

namespace jp {

// classical iff OUT_J < ratio * (|R| + |S|) (JP_F1_RATIO overrides)
constexpr double JP_F1_RATIO_DEFAULT = 1.0;
// most join rows the classical path takes (its dedup set holds 2^31 slots at most)
constexpr int64_t JP_CLASSICAL_MAX_OUT_J = int64_t(1) << 30;

// OUT_J estimated from up to 4096 sampled tuples per side (exact below that); syncs
int64_t estimate_out_j(const int32_t* ry, int64_t nr, const int32_t* sy, int64_t ns, hipStream_t s);
// the same in two halves: the sample's matching pairs into *matches (device, asynchronous), then the estimate
void launch_out_j_sample(const int32_t* ry, int64_t nr, const int32_t* sy, int64_t ns, unsigned long long* matches,
                         hipStream_t s);
int64_t out_j_from_sample(unsigned long long matches, int64_t nr, int64_t ns);
bool f1_prefers_classical(int64_t out_j_est, int64_t nr, int64_t ns);

struct ClassicalPlan {
  Budget B;
  Arena A{&B};
  hipStream_t stream = nullptr;
  const int32_t* rx = nullptr;
  int64_t nr = 0, ns = 0;
  // build side: open-addressing table on S.y (cap_s slots), S.z grouped by slot
  int shift_s = 63;
  int64_t cap_s = 0;
  int64_t* skey = nullptr;
  int32_t *start = nullptr, *zlist = nullptr;
  // probe side
  int64_t *rslot = nullptr, *jr_off = nullptr;
  int64_t out_j = 0, n_x = 0, n_y = 0, n_z = 0, n_r_kept = 0;
  // deduplication set of 64-bit pair keys
  int shift_d = 63;
  int64_t cap_d = 0;
  uint64_t* set = nullptr;
  unsigned long long* d_cnt = nullptr;
  int32_t* d_extra = nullptr;
  bool executed = false, have_total = false, sorted = false;
  int64_t total = 0;
  // sorted result and its rows (built at the first materialise or row query)
  int32_t *sx = nullptr, *sz_ = nullptr, *xv = nullptr;
  int64_t* xoff = nullptr;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

  ~ClassicalPlan();
  bool timing_on() const { return ev[0] != nullptr; }
  void arena_limit(int64_t lim) { B.limit = lim; }
  void build(const int32_t* rx, const int32_t* ry, int64_t nr, const int32_t* sz, const int32_t* sy, int64_t ns,
             bool timing, hipStream_t s);
  void execute(hipStream_t s);
  void fetch_total(hipStream_t s);
  void sort_result(hipStream_t s);
  int64_t materialize(int part, int64_t first, int64_t maxp, int32_t* ox, int32_t* oz, hipStream_t s);
  void row_info(int part, int32_t* x_values, int64_t* row_offsets, hipStream_t s);
  void stats(jp_stats* st) const;
  void timings(jp_timings* t, hipStream_t s);
};

}  // namespace jp
