// Query server behind jp_server_* (include/jp.h): continuous batching of
// Join-Project queries on one GPU.
//
// One host thread owns two streams.  Each turn it admits the queued queries
// whose estimated device footprint fits what the HBM budget leaves beside the
// batches still in flight, plans them as one batch (all stages one launch over
// all of them) and runs the count pass.  While that batch runs on one stream,
// the next turn plans the queries that arrived meanwhile on the other stream,
// so planning (host read-backs included) overlaps execution.  At most two
// batches are in flight; a finished batch's counts go to its queries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
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

using namespace jp;

namespace {

struct Query {
  jp_instance inst{};
  int64_t est = 0;
  jp_query_result res{};
  bool done = false;
};

struct InFlight {
  std::unique_ptr<Plan> plan;
  std::vector<uint64_t> ids;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  int64_t bytes = 0;
};

// device bytes a query is expected to need: sort buffers, CSR, partition and
// dense structures grow with the tuple counts
int64_t estimate_bytes(const jp_instance& q) { return 96 * (q.n_r + q.n_s) + (int64_t(1) << 20); }

}  // namespace

struct jp_server {
  jp_server_config cfg{};
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Query> queries;
  uint64_t next_id = 1;
  bool stopping = false;
  int64_t inflight_bytes = 0;
  jp_server_summary st{};
  std::vector<double> lat;
  std::thread th;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
  }

  void finish(const std::vector<uint64_t>& ids, const Plan* plan, int status) {
    std::lock_guard<std::mutex> g(mu);
    const double t = now_us();
    for (size_t i = 0; i < ids.size(); ++i) {
      Query& q = queries[ids[i]];
      q.res.status = status;
      q.res.batch_size = int32_t(ids.size());
      if (status == JP_OK) {
        q.res.total = plan->h_tot[3 * i + 0];
        q.res.dense = plan->h_tot[3 * i + 1];
        q.res.sparse = plan->h_tot[3 * i + 2];
        st.completed += 1;
        st.pairs += q.res.total;
      } else {
        st.failed += 1;
      }
      q.res.done_us = t;
      q.done = true;
      lat.push_back(t - q.res.submit_us);
    }
    cv_done.notify_all();
  }

  void loop() {
    (void)hipSetDevice(cfg.device);
    hipStream_t streams[2];
    for (auto& s : streams) (void)hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    std::deque<InFlight> inflight;
    int turn = 0;
    const int64_t budget = cfg.hbm_budget_bytes > 0 ? cfg.hbm_budget_bytes : (int64_t(64) << 30);
    const size_t max_batch = cfg.max_batch > 0 ? size_t(cfg.max_batch) : 4096;
    while (true) {
      // retire the batches that have finished
      while (!inflight.empty() && hipEventQuery(inflight.front().ev) == hipSuccess) retire(inflight);
      std::vector<uint64_t> take;
      std::vector<uint64_t> too_big;
      {
        std::unique_lock<std::mutex> lk(mu);
        if (stopping && pending.empty() && inflight.empty()) break;
        if (inflight.size() < 2) {
          int64_t left = budget - inflight_bytes;
          while (!pending.empty() && take.size() < max_batch) {
            Query& q = queries[pending.front()];
            if (q.est > budget) {  // can never fit: fail it
              too_big.push_back(pending.front());
              pending.pop_front();
              continue;
            }
            if (q.est > left) break;
            left -= q.est;
            q.res.admit_us = now_us();
            take.push_back(pending.front());
            pending.pop_front();
          }
        }
      }
      if (!too_big.empty()) finish(too_big, nullptr, JP_ENOMEM);
      if (!take.empty()) {
        InFlight f;
        f.ids = take;
        f.stream = streams[turn];
        turn ^= 1;
        std::vector<jp_instance> inst;
        int64_t est = 0;
        {
          std::lock_guard<std::mutex> g(mu);
          for (uint64_t id : take) {
            inst.push_back(queries[id].inst);
            est += queries[id].est;
          }
          inflight_bytes += est;
        }
        f.bytes = est;
        f.plan.reset(new Plan());
        int status = JP_OK;
        try {
          f.plan->build(inst.data(), int(inst.size()), &cfg.opt, f.stream);
          f.plan->execute(f.stream);
          if (hipEventCreateWithFlags(&f.ev, hipEventDisableTiming) != hipSuccess ||
              hipEventRecord(f.ev, f.stream) != hipSuccess)
            throw Error(JP_EHIP, "event record failed");
        } catch (const Error& e) {
          status = e.status;
        } catch (...) {
          status = JP_EHIP;
        }
        {
          std::lock_guard<std::mutex> g(mu);
          st.batches += 1;
          // the plan's real footprint replaces the estimate
          inflight_bytes += f.plan->A.bytes() - est;
          f.bytes = f.plan->A.bytes();
          st.peak_bytes = std::max(st.peak_bytes, inflight_bytes);
        }
        if (status != JP_OK) {
          (void)hipStreamSynchronize(f.stream);
          finish(f.ids, nullptr, status);
          release(f);
        } else {
          inflight.push_back(std::move(f));
        }
        continue;  // plan the next arrivals while this batch runs
      }
      if (!too_big.empty()) continue;
      // nothing to launch now
      if (inflight.empty()) {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stopping || !pending.empty(); });
        continue;
      }
      bool waiting_room;
      {
        std::lock_guard<std::mutex> g(mu);
        // queries are queued but do not fit: only a finished batch frees room
        waiting_room = inflight.size() >= 2 || !pending.empty();
      }
      if (waiting_room) {
        (void)hipEventSynchronize(inflight.front().ev);
      } else {
        // GPU busy, queue empty: wake on a new arrival or poll the batch soon
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait_for(lk, std::chrono::microseconds(50), [&] { return stopping || !pending.empty(); });
      }
    }
    for (auto& s : streams) (void)hipStreamDestroy(s);
  }

  void retire(std::deque<InFlight>& inflight) {
    InFlight& f = inflight.front();
    int status = JP_OK;
    try {
      f.plan->fetch_totals(f.stream);
    } catch (const Error& e) {
      status = e.status;
    }
    finish(f.ids, f.plan.get(), status);
    release(f);
    inflight.pop_front();
  }

  void release(InFlight& f) {
    if (f.ev) (void)hipEventDestroy(f.ev);
    f.ev = nullptr;
    const int64_t b = f.bytes;
    f.plan.reset();  // returns its memory to the pool (stream-ordered)
    std::lock_guard<std::mutex> g(mu);
    inflight_bytes -= b;
  }
};

namespace {
jp_status sfail(int st, const char* m) {
  jp::set_last_error(m);
  return jp_status(st);
}
}  // namespace

extern "C" {

jp_status jp_server_create(const jp_server_config* cfg, jp_server** out) {
  if (!cfg || !out) return sfail(JP_EINVAL, "null argument");
  if (cfg->max_batch < 0 || cfg->hbm_budget_bytes < 0) return sfail(JP_EINVAL, "negative limit");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || cfg->device < 0 || cfg->device >= n)
    return sfail(JP_EINVAL, "bad device");
  jp_server* s = new (std::nothrow) jp_server();
  if (!s) return sfail(JP_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  s->t0 = std::chrono::steady_clock::now();
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
  qq.est = estimate_bytes(*q);
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

jp_status jp_server_stats(jp_server* s, jp_server_summary* out) {
  if (!s || !out) return sfail(JP_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->st;
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
  delete s;
}

}  // extern "C"
