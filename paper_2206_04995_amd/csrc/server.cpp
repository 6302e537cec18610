// Query server behind jp_server_* (include/jp.h): continuous batching of
// Join-Project queries on one GPU.
//
// One host thread owns two streams.  Each turn it admits the queued queries
// whose estimated device footprint fits what the HBM budget leaves beside the
// batches still in flight (or kept), plans them as one batch (all stages one
// launch over all of them) and runs the count pass.  While that batch runs on
// one stream, the next turn plans the queries that arrived meanwhile on the
// other stream, so planning (host read-backs included) overlaps execution.  At
// most two batches are in flight; a finished batch's counts (and, on request,
// digests) go to its queries.
//
// Footprint accounting.  A query's estimate covers its plan (mapping, CSR,
// partition and count-pass state, temporaries included: a fixed number of
// bytes per input tuple) and its output: pairs of one materialised chunk of
// at most min(n_r * n_s, chunk_pairs) pairs when digests are computed or the
// result is kept.  A batch is planned with its summed estimate as the limit
// of every device byte its plan holds at once, so the batches admitted
// together never hold more than the budget.  A batch that fails is split in
// halves and planned again, so one query's failure (a value range that does
// not stack with the others', a footprint above its estimate) stays its own;
// a single query above its estimate is retried once alone with everything the
// budget leaves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/jp.h"
#include "plan_impl.h"
#include "prim.h"

using namespace jp;

namespace {

// device bytes per input tuple a plan may hold at once (sort buffers, CSR,
// partition tables, count pass, temporaries), and a fixed part per query
constexpr int64_t EST_BYTES_PER_TUPLE = 160;
constexpr int64_t EST_FIXED_BYTES = int64_t(2) << 20;
constexpr int64_t DEFAULT_CHUNK_PAIRS = int64_t(1) << 24;

struct BatchState;

struct Query {
  jp_instance inst{};
  int64_t est = 0;
  bool solo_tried = false;  // already retried alone with the whole free budget
  int index = -1;           // position in its batch
  jp_query_result res{};
  bool done = false;
  std::shared_ptr<BatchState> batch;  // set while the result is kept
};

}  // namespace

struct jp_server;

namespace {

// One planned batch.  Shared by the in-flight list and by the kept queries;
// its device memory and its budget charge go when the last owner drops it.
struct BatchState {
  jp_server* srv = nullptr;
  std::unique_ptr<Plan> plan;
  std::vector<uint64_t> ids;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  int64_t charge = 0;
  bool kept = false;  // its results are kept (its peak counts in kept_peak)
  std::mutex mu;      // one materialisation at a time on the plan
  ~BatchState();
};

}  // namespace

struct jp_server {
  jp_server_config cfg{};
  int64_t budget = 0;
  int64_t chunk = DEFAULT_CHUNK_PAIRS;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Query> queries;
  uint64_t next_id = 1;
  bool stopping = false;
  int64_t charged = 0;      // budget charges of live batches (in flight or kept)
  int64_t live_peak = 0;    // sum over live batches of their peak device bytes
  jp_server_summary st{};
  std::vector<double> lat;
  hipStream_t streams[2] = {nullptr, nullptr};
  std::vector<std::shared_ptr<BatchState>> live;  // in flight (server thread only)
  std::thread th;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }

  int64_t estimate(const jp_instance& q) const {
    int64_t est = EST_BYTES_PER_TUPLE * (q.n_r + q.n_s) + EST_FIXED_BYTES;
    if (cfg.flags & (JP_SERVER_DIGEST | JP_SERVER_KEEP)) {
      // one chunk of output pairs: the chunk buffers and the write pass's row lists
      const double bound = double(q.n_r) * double(q.n_s);
      const int64_t pairs = bound < double(chunk) ? int64_t(bound) : chunk;
      est += 16 * pairs;
    }
    return est;
  }

  // results of one query (under mu)
  void finish_one(uint64_t id, int status, const int64_t* tot, const uint64_t* digest, int batch_size,
                  const std::shared_ptr<BatchState>& keep) {
    Query& q = queries[id];
    q.res.status = status;
    q.res.batch_size = batch_size;
    if (status == JP_OK) {
      q.res.total = tot[0];
      q.res.dense = tot[1];
      q.res.sparse = tot[2];
      q.res.has_digest = digest ? 1 : 0;
      q.res.digest = digest ? *digest : 0;
      q.res.kept = keep ? 1 : 0;
      q.batch = keep;
      st.completed += 1;
      st.pairs += q.res.total;
    } else {
      st.failed += 1;
    }
    q.res.done_us = now_us();
    q.done = true;
    lat.push_back(q.res.done_us - q.res.submit_us);
  }

  void fail_all(const std::vector<uint64_t>& ids, int status) {
    std::lock_guard<std::mutex> g(mu);
    for (uint64_t id : ids) finish_one(id, status, nullptr, nullptr, int(ids.size()), nullptr);
    cv_done.notify_all();
  }

  // Takes the next group of queries that fits beside the live batches.
  // Returns the group and its charge (empty when nothing can go now).
  std::vector<uint64_t> admit(int64_t* charge, std::vector<uint64_t>* too_big) {
    std::vector<uint64_t> take;
    *charge = 0;
    std::lock_guard<std::mutex> g(mu);
    if (pending.empty() || live.size() >= 2) return take;
    // after a split, the next group is the first half at the front of the queue
    const size_t max_batch = split_cap > 0 ? split_cap : (cfg.max_batch > 0 ? size_t(cfg.max_batch) : 4096);
    split_cap = 0;
    int64_t left = budget - charged, sum_r = 0, sum_s = 0;
    Query& head = queries[pending.front()];
    if (head.solo_tried) {
      // alone, with everything the budget leaves once no batch is in flight
      if (!live.empty()) return take;
      if (left <= head.est) {  // nothing more to give than its failed attempt had
        too_big->push_back(pending.front());
        pending.pop_front();
        return take;
      }
      head.res.admit_us = now_us();
      take.push_back(pending.front());
      pending.pop_front();
      *charge = left;
      return take;
    }
    while (!pending.empty() && take.size() < max_batch) {
      Query& q = queries[pending.front()];
      if (q.solo_tried) break;
      if (q.est > budget) {  // can never fit: fail it
        too_big->push_back(pending.front());
        pending.pop_front();
        continue;
      }
      if (q.est > left || sum_r + q.inst.n_r > INT32_MAX || sum_s + q.inst.n_s > INT32_MAX) break;
      left -= q.est;
      sum_r += q.inst.n_r;
      sum_s += q.inst.n_s;
      *charge += q.est;
      q.res.admit_us = now_us();
      take.push_back(pending.front());
      pending.pop_front();
    }
    return take;
  }

  // Plans and launches one group; on failure splits it (or fails a single query).
  void launch(std::vector<uint64_t> ids, int64_t charge, hipStream_t s) {
    auto b = std::make_shared<BatchState>();
    b->srv = this;
    b->ids = ids;
    b->stream = s;
    b->charge = charge;
    std::vector<jp_instance> inst;
    {
      std::lock_guard<std::mutex> g(mu);
      for (size_t i = 0; i < ids.size(); ++i) {
        Query& q = queries[ids[i]];
        q.index = int(i);
        inst.push_back(q.inst);
      }
      charged += charge;
    }
    b->plan.reset(new Plan());
    int status = JP_OK;
    std::string msg;
    try {
      jp_options o = cfg.opt;
      o.workspace_limit_bytes = charge;
      b->plan->build(inst.data(), int(inst.size()), &o, s);
      b->plan->execute(s);
      JP_HIP(hipEventCreateWithFlags(&b->ev, hipEventDisableTiming));
      JP_HIP(hipEventRecord(b->ev, s));
    } catch (const Error& e) {
      status = e.status;
      msg = e.what();
    } catch (...) {
      status = JP_EHIP;
    }
    {
      std::lock_guard<std::mutex> g(mu);
      st.batches += 1;
    }
    if (status == JP_OK) {
      live.push_back(b);
      note_peak();
      return;
    }
    (void)hipStreamSynchronize(s);
    b.reset();  // frees the plan and its charge
    std::lock_guard<std::mutex> g(mu);
    if (ids.size() > 1) {
      // split: both halves go back to the front of the queue, in order, and
      // the next admission takes the first half alone
      for (size_t i = ids.size(); i-- > 0;) pending.push_front(ids[i]);
      st.splits += 1;
      split_cap = ids.size() / 2;
    } else if (status == JP_ENOMEM && !queries[ids[0]].solo_tried) {
      queries[ids[0]].solo_tried = true;
      pending.push_front(ids[0]);
    } else {
      finish_one(ids[0], status, nullptr, nullptr, 1, nullptr);
      cv_done.notify_all();
    }
  }

  size_t split_cap = 0;  // > 0: size of the next group (a split half; under mu)

  void note_peak() {
    int64_t sum = 0;
    for (auto& b : live) sum += b->plan->B.peak;
    std::lock_guard<std::mutex> g(mu);
    live_peak = sum + kept_peak;
    st.peak_bytes = std::max(st.peak_bytes, live_peak);
  }
  int64_t kept_peak = 0;  // peak bytes of kept batches (under mu)

  // Counts (and digests) of a finished batch go to its queries.
  void retire() {
    std::shared_ptr<BatchState> b = live.front();
    live.erase(live.begin());
    int status = JP_OK;
    std::vector<uint64_t> dig;
    try {
      b->plan->fetch_totals(b->stream);
      if (cfg.flags & JP_SERVER_DIGEST) dig = digests(*b);
    } catch (const Error& e) {
      status = e.status;
    } catch (...) {
      status = JP_EHIP;
    }
    note_peak();
    const bool keep = status == JP_OK && (cfg.flags & JP_SERVER_KEEP);
    {
      std::lock_guard<std::mutex> g(mu);
      for (size_t i = 0; i < b->ids.size(); ++i)
        finish_one(b->ids[i], status, status == JP_OK ? &b->plan->h_tot[3 * i] : nullptr,
                   dig.empty() ? nullptr : &dig[i], int(b->ids.size()), keep ? b : nullptr);
      if (keep) {
        b->kept = true;
        kept_peak += b->plan->B.peak;
      }
      cv_done.notify_all();
    }
    b.reset();  // dropped here unless kept
  }

  // Order-independent digest of each query's pairs: chunks of the sorted
  // result are materialised into plan-owned buffers and digested on the device.
  std::vector<uint64_t> digests(BatchState& b) {
    Plan& p = *b.plan;
    const int n = p.n_inst;
    int64_t most = 0;
    for (int i = 0; i < n; ++i) most = std::max(most, p.h_tot[3 * size_t(i)]);
    const int64_t cap = std::max<int64_t>(1, std::min(most, chunk));
    int32_t* bx = p.A.alloc<int32_t>(cap, b.stream);
    int32_t* bz = p.A.alloc<int32_t>(cap, b.stream);
    uint64_t* acc = p.A.alloc<uint64_t>(n, b.stream);
    fill_i64(reinterpret_cast<int64_t*>(acc), n, 0, b.stream);
    for (int i = 0; i < n; ++i) {
      const int64_t total = p.h_tot[3 * size_t(i)];
      for (int64_t first = 0; first < total; first += cap) {
        const int64_t w = p.materialize(i, JP_PART_ALL, first, cap, bx, bz, b.stream);
        digest_pairs(bx, bz, w, acc + i, b.stream);
      }
    }
    std::vector<uint64_t> out(n);
    JP_HIP(hipMemcpyAsync(out.data(), acc, n * sizeof(uint64_t), hipMemcpyDeviceToHost, b.stream));
    JP_HIP(hipStreamSynchronize(b.stream));
    p.A.give_back(bx, b.stream);
    p.A.give_back(bz, b.stream);
    p.A.give_back(acc, b.stream);
    return out;
  }

  void loop() {
    (void)hipSetDevice(cfg.device);
    int turn = 0;
    while (true) {
      while (!live.empty() && hipEventQuery(live.front()->ev) == hipSuccess) retire();
      int64_t charge = 0;
      std::vector<uint64_t> too_big;
      std::vector<uint64_t> take = admit(&charge, &too_big);
      if (!too_big.empty()) fail_all(too_big, JP_ENOMEM);
      if (!take.empty()) {
        launch(take, charge, streams[turn]);
        turn ^= 1;
        continue;  // plan the next arrivals while this batch runs
      }
      if (!too_big.empty()) continue;
      bool idle_stop, waiting_room;
      {
        std::lock_guard<std::mutex> g(mu);
        idle_stop = stopping && pending.empty() && live.empty();
        // queries are queued but cannot go: only a finished batch frees room
        waiting_room = !pending.empty();
      }
      if (idle_stop) break;
      if (live.empty()) {
        std::unique_lock<std::mutex> lk(mu);
        if (!pending.empty()) {
          // queued but blocked by kept results only: wait for a release
          cv_work.wait_for(lk, std::chrono::milliseconds(1));
        } else {
          cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
        }
        continue;
      }
      if (waiting_room || live.size() >= 2) {
        (void)hipEventSynchronize(live.front()->ev);
      } else {
        // GPU busy, queue empty: wake on a new arrival or poll the batch soon
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return stopping || !pending.empty(); });
      }
    }
  }
};

namespace {

BatchState::~BatchState() {
  const int64_t peak = plan ? plan->B.peak : 0;
  if (ev) (void)hipEventDestroy(ev);
  plan.reset();  // returns its memory to the pool (stream-ordered)
  if (srv) {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->charged -= charge;
    if (kept) srv->kept_peak -= peak;
  }
}

jp_status sfail(int st, const std::string& m) {
  jp::set_last_error(m);
  return jp_status(st);
}

}  // namespace

extern "C" {

jp_status jp_server_create(const jp_server_config* cfg, jp_server** out) {
  if (!cfg || !out) return sfail(JP_EINVAL, "null argument");
  *out = nullptr;
  if (cfg->max_batch < 0 || cfg->hbm_budget_bytes < 0 || cfg->chunk_pairs < 0)
    return sfail(JP_EINVAL, "negative limit");
  if (cfg->flags & ~(JP_SERVER_DIGEST | JP_SERVER_KEEP)) return sfail(JP_EINVAL, "unknown server flag bits");
  if (cfg->reserved != 0) return sfail(JP_EINVAL, "reserved server field must be 0");
  if (cfg->opt.flags & (JP_FLAG_TIMING | JP_FLAG_GRAPH))
    return sfail(JP_EINVAL, "server options take neither JP_FLAG_TIMING nor JP_FLAG_GRAPH");
  jp_status st = jp::check_options(&cfg->opt);
  if (st != JP_OK) return st;
  if (cfg->opt.strategy == JP_STRATEGY_CLASSICAL)
    return sfail(JP_EINVAL, "the server runs the hybrid path (JP_STRATEGY_CLASSICAL is for single plans)");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || cfg->device < 0 || cfg->device >= n)
    return sfail(JP_EINVAL, "bad device");
  jp_server* s = new (std::nothrow) jp_server();
  if (!s) return sfail(JP_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->budget = cfg->hbm_budget_bytes > 0 ? cfg->hbm_budget_bytes : (int64_t(64) << 30);
  s->chunk = cfg->chunk_pairs > 0 ? cfg->chunk_pairs : DEFAULT_CHUNK_PAIRS;
  s->t0 = std::chrono::steady_clock::now();
  int prev = 0;
  (void)hipGetDevice(&prev);
  bool ok = hipSetDevice(cfg->device) == hipSuccess;
  for (auto& q : s->streams) ok = ok && hipStreamCreateWithFlags(&q, hipStreamNonBlocking) == hipSuccess;
  (void)hipSetDevice(prev);
  if (!ok) {
    for (auto& q : s->streams)
      if (q) (void)hipStreamDestroy(q);
    delete s;
    return sfail(JP_EHIP, "stream creation failed");
  }
  s->th = std::thread([s] { s->loop(); });
  *out = s;
  return JP_OK;
}

jp_status jp_server_submit(jp_server* s, const jp_instance* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return sfail(JP_EINVAL, "null argument");
  if (q->n_r < 0 || q->n_s < 0 || q->n_r > INT32_MAX || q->n_s > INT32_MAX) return sfail(JP_EINVAL, "bad tuple count");
  if ((q->n_r > 0 && (!q->r_x || !q->r_y)) || (q->n_s > 0 && (!q->s_z || !q->s_y)))
    return sfail(JP_EINVAL, "null column with n > 0");
  std::lock_guard<std::mutex> g(s->mu);
  if (s->stopping) return sfail(JP_EBUSY, "server is stopping");
  const uint64_t id = s->next_id++;
  Query& qq = s->queries[id];
  qq.inst = *q;
  qq.est = s->estimate(*q);
  qq.res.submit_us = s->now_us();
  s->pending.push_back(id);
  s->st.submitted += 1;
  *ticket = id;
  s->cv_work.notify_one();
  return JP_OK;
}

jp_status jp_server_poll(jp_server* s, uint64_t ticket, int* done, jp_query_result* r) {
  if (!s || !done) return sfail(JP_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->queries.find(ticket);
  if (it == s->queries.end()) return sfail(JP_EINVAL, "unknown ticket");
  *done = it->second.done ? 1 : 0;
  if (it->second.done && r) *r = it->second.res;
  return JP_OK;
}

jp_status jp_server_wait(jp_server* s, uint64_t ticket, jp_query_result* r) {
  if (!s) return sfail(JP_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->queries.find(ticket);
  if (it == s->queries.end()) return sfail(JP_EINVAL, "unknown ticket");
  s->cv_done.wait(lk, [&] { return s->queries[ticket].done; });
  if (r) *r = s->queries[ticket].res;
  return JP_OK;
}

jp_status jp_server_materialize(jp_server* s, uint64_t ticket, jp_part part, int64_t first, int64_t max_pairs,
                                int32_t* out_x, int32_t* out_z, int64_t* n_written, hipStream_t stream) {
  if (!s || !n_written) return sfail(JP_EINVAL, "null argument");
  if (part < JP_PART_ALL || part > JP_PART_SPARSE) return sfail(JP_EINVAL, "bad part");
  if (first < 0 || max_pairs < 0) return sfail(JP_EINVAL, "negative first or max_pairs");
  if (max_pairs > 0 && (!out_x || !out_z)) return sfail(JP_EINVAL, "null output with max_pairs > 0");
  *n_written = 0;
  std::shared_ptr<BatchState> b;
  int index = -1;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return sfail(JP_EINVAL, "unknown ticket");
    if (!it->second.done || !it->second.batch)
      return sfail(JP_ESTATE, "the result is not kept (not done, failed, released, or the server lacks JP_SERVER_KEEP)");
    b = it->second.batch;
    index = it->second.index;
  }
  std::lock_guard<std::mutex> g(b->mu);
  try {
    *n_written = b->plan->materialize(index, int(part), first, max_pairs, out_x, out_z, stream);
  } catch (const Error& e) {
    return sfail(e.status, e.what());
  } catch (...) {
    return sfail(JP_EHIP, "materialisation failed");
  }
  return JP_OK;
}

jp_status jp_server_release(jp_server* s, uint64_t ticket) {
  if (!s) return sfail(JP_EINVAL, "null argument");
  std::shared_ptr<BatchState> drop;
  {
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->queries.find(ticket);
    if (it == s->queries.end()) return sfail(JP_EINVAL, "unknown ticket");
    if (!it->second.done) return sfail(JP_ESTATE, "the query is not done");
    drop = std::move(it->second.batch);
    it->second.res.kept = 0;
  }
  drop.reset();  // the batch goes once its last kept query is released
  s->cv_work.notify_all();
  return JP_OK;
}

jp_status jp_server_stats(jp_server* s, jp_server_summary* out) {
  if (!s || !out) return sfail(JP_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
  out->budget_bytes = s->budget;
  out->charged_bytes = s->charged;
  if (!s->lat.empty()) {
    std::vector<double> v = s->lat;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) { return v[std::min(v.size() - 1, size_t(p * double(v.size() - 1) + 0.5))]; };
    out->p50_us = pct(0.50);
    out->p99_us = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_us = sum / double(v.size());
  }
  return JP_OK;
}

void jp_server_destroy(jp_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stopping = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  std::vector<std::shared_ptr<BatchState>> kept;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (auto& kv : s->queries)
      if (kv.second.batch) kept.push_back(std::move(kv.second.batch));
  }
  kept.clear();  // kept plans go before their streams
  for (auto& q : s->streams)
    if (q) {
      (void)hipStreamSynchronize(q);
      (void)hipStreamDestroy(q);
    }
  delete s;
}

}  // extern "C"
