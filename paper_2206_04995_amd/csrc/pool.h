// Caching device allocator and error plumbing for the Join-Project library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

namespace jp {

// Error carried from a failing step to the C ABI boundary (never crosses it).
struct Error : std::runtime_error {
  int status;
  Error(int st, const std::string& m) : std::runtime_error(m), status(st) {}
};

#define JP_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::jp::Error(3, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

#define JP_LAUNCH_CHECK() JP_HIP(hipGetLastError())

// Device memory cache.  Blocks freed on a stream are reused at once by the
// same stream (stream order makes that safe) and by other streams only after
// an event recorded at the free has completed.  Memory is returned to HIP only
// by trim() or at process exit.
class Pool {
 public:
  static Pool& instance();
  void* alloc(size_t bytes, hipStream_t s);
  void free(void* p, hipStream_t s);
  void trim();
  size_t cached_bytes() const { return cached_; }

 private:
  struct Block {
    void* p;
    size_t size;
    hipStream_t stream;
    hipEvent_t ev;
    int device;
  };
  std::mutex mu_;
  std::multimap<size_t, Block> free_;
  std::map<void*, Block> used_;
  size_t cached_ = 0;
};

// A fixed device region that arenas carve their blocks from, instead of the
// pool, while a RegionScope is active on the calling thread: blocks are taken
// in order (256-byte aligned) and none is returned before the scope ends, so
// the region must hold everything the work of the scope allocates.  Running
// out throws JP_ENOMEM.
struct Region {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
};
Region* active_region();  // of the calling thread; null outside any scope
class RegionScope {
 public:
  explicit RegionScope(Region* r);
  ~RegionScope();
  RegionScope(const RegionScope&) = delete;
  RegionScope& operator=(const RegionScope&) = delete;

 private:
  Region* prev_;
};

// Device bytes held at once by every arena of one owner (a plan: its
// persistent state and its temporaries), checked against an optional limit.
struct Budget {
  int64_t limit = 0;  // 0: none
  int64_t used = 0;
  int64_t peak = 0;
};

// Allocation owner: returns everything to the pool on release().  Every block
// is charged to the owner's budget (if any); a block that would take the
// budget past its limit throws JP_ENOMEM before anything is allocated.
class Arena {
 public:
  explicit Arena(Budget* b = nullptr) : budget_(b) {}
  ~Arena() { release(nullptr); }
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;

  template <class T>
  T* alloc(int64_t count, hipStream_t s) {
    return static_cast<T*>(raw(size_t(count < 1 ? 1 : count) * sizeof(T), s));
  }
  void* raw(size_t bytes, hipStream_t s);
  void give_back(void* p, hipStream_t s);  // return one block early
  void release(hipStream_t s);
  int64_t bytes() const { return bytes_; }

  // Replay mode: the first pass records its allocations and keeps them
  // (give_back does nothing); every later pass, started by rewind(), gets the
  // same blocks in the same order without touching the allocator, so the
  // pass can be captured into a graph or run where allocation is not allowed.
  void set_replay(bool on) { replay_ = on; }
  void rewind() { cursor_ = 0; }

 private:
  struct Rec {
    void* p;
    size_t bytes;
  };
  void charge(int64_t b);
  std::vector<Rec> recs_;
  Budget* budget_;
  int64_t bytes_ = 0;
  bool replay_ = false;
  size_t cursor_ = 0;
};

inline size_t round_alloc(size_t b) {
  if (b <= 4096) return 4096;
  if (b <= (1u << 20)) return (b + 4095) & ~size_t(4095);
  return (b + (size_t(1) << 20) - 1) & ~((size_t(1) << 20) - 1);
}

}  // namespace jp
