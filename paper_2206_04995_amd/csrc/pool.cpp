// Caching device allocator (see pool.h).
#include "pool.h"

namespace jp {

Pool& Pool::instance() {
  static Pool* p = new Pool();  // leaked on purpose: outlives every plan
  return *p;
}

void* Pool::alloc(size_t bytes, hipStream_t s) {
  size_t want = round_alloc(bytes);
  int dev = 0;
  JP_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(mu_);
    // best fit among blocks no larger than 1.25x the request
    auto it = free_.lower_bound(want);
    while (it != free_.end() && it->first <= want + want / 4) {
      Block& b = it->second;
      bool ok = b.device == dev && (b.stream == s || hipEventQuery(b.ev) == hipSuccess);
      if (ok) {
        Block blk = b;
        free_.erase(it);
        cached_ -= blk.size;
        used_[blk.p] = blk;
        return blk.p;
      }
      ++it;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // give cached memory back and try once more
    trim();
    e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw Error(2, "device allocation of " + std::to_string(want) + " bytes failed");
    }
  }
  Block blk{p, want, s, nullptr, dev};
  JP_HIP(hipEventCreateWithFlags(&blk.ev, hipEventDisableTiming));
  std::lock_guard<std::mutex> g(mu_);
  used_[p] = blk;
  return p;
}

void Pool::free(void* p, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  auto it = used_.find(p);
  if (it == used_.end()) return;
  Block b = it->second;
  used_.erase(it);
  b.stream = s;
  if (hipEventRecord(b.ev, s) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipDeviceSynchronize();
  }
  free_.emplace(b.size, b);
  cached_ += b.size;
}

void Pool::trim() {
  std::vector<Block> drop;
  {
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end();) {
      if (hipEventQuery(it->second.ev) == hipSuccess) {
        drop.push_back(it->second);
        cached_ -= it->second.size;
        it = free_.erase(it);
      } else {
        ++it;
      }
    }
  }
  for (auto& b : drop) {
    (void)hipEventDestroy(b.ev);
    (void)hipFree(b.p);
  }
}

namespace {
thread_local Region* t_region = nullptr;
}

Region* active_region() { return t_region; }
RegionScope::RegionScope(Region* r) : prev_(t_region) { t_region = r; }
RegionScope::~RegionScope() { t_region = prev_; }

void Arena::charge(int64_t b) {
  if (budget_) {
    if (budget_->limit > 0 && budget_->used + b > budget_->limit)
      throw Error(2, "workspace limit of " + std::to_string(budget_->limit) + " bytes exceeded");
    budget_->used += b;
    if (budget_->used > budget_->peak) budget_->peak = budget_->used;
  }
  bytes_ += b;
}

void* Arena::raw(size_t bytes, hipStream_t s) {
  if (Region* g = t_region) {
    // carved from the caller's fixed region: never recorded, never freed
    const size_t r = bytes == 0 ? 256 : (bytes + 255) & ~size_t(255);
    if (r > g->size - g->used)
      throw Error(2, "the query needs more than the " + std::to_string(g->size) + " bytes of the static scratch");
    charge(int64_t(r));
    void* p = g->base + g->used;
    g->used += r;
    return p;
  }
  size_t r = round_alloc(bytes);
  if (replay_ && cursor_ < recs_.size()) {
    Rec& rec = recs_[cursor_];
    if (rec.bytes < r) throw Error(4, "replayed allocation sequence changed");
    ++cursor_;
    return rec.p;
  }
  charge(int64_t(r));
  void* p = nullptr;
  try {
    p = Pool::instance().alloc(bytes, s);
  } catch (...) {
    bytes_ -= int64_t(r);
    if (budget_) budget_->used -= int64_t(r);
    throw;
  }
  recs_.push_back({p, r});
  if (replay_) cursor_ = recs_.size();
  return p;
}

void Arena::give_back(void* p, hipStream_t s) {
  if (replay_) return;  // kept for the next pass
  for (size_t i = 0; i < recs_.size(); ++i) {
    if (recs_[i].p == p) {
      bytes_ -= int64_t(recs_[i].bytes);
      if (budget_) budget_->used -= int64_t(recs_[i].bytes);
      Pool::instance().free(p, s);
      recs_[i] = recs_.back();
      recs_.pop_back();
      return;
    }
  }
}

void Arena::release(hipStream_t s) {
  for (auto& r : recs_) Pool::instance().free(r.p, s);
  recs_.clear();
  if (budget_) budget_->used -= bytes_;
  bytes_ = 0;
  cursor_ = 0;
}

}  // namespace jp
