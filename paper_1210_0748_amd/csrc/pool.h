// Process-wide caching allocator for device memory.
//
// A job allocates and frees a few GB of buffers; going to hipMalloc/hipFree
// each time costs milliseconds and an implicit device synchronisation. Freed
// blocks are kept per device and handed out again (best fit, at most twice
// the requested size). A block remembers the stream of its last user through
// an event: a later user on another stream makes its stream wait for that
// event, so reuse is ordered after every kernel that touched the block. When hipMalloc
// fails, all cached blocks are released and the allocation is retried.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.h"

namespace kb {

// A fixed device region that serves every allocation of the calling thread
// while an ArenaScope is active (first fit, neighbours merged on free). The
// library's allocation-free entry point runs a whole job inside one; all its
// work is on one stream, so a block freed there can be reused by the next
// allocation at once (later kernels are ordered after earlier ones).
class Arena {
 public:
  Arena(void* base, size_t bytes) : base_(static_cast<char*>(base)), bytes_(bytes) { free_[0] = bytes; }
  void* get(size_t want) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < want) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > want) free_[off + want] = len - want;
      used_ += want;
      peak_ = used_ > peak_ ? used_ : peak_;
      return base_ + off;
    }
    throw OutOfMemory("the static scratch region (" + std::to_string(bytes_) + " bytes) is exhausted");
  }
  bool owns(const void* p) const {
    const char* c = static_cast<const char*>(p);
    return c >= base_ && c < base_ + bytes_;
  }
  void put(void* p, size_t bytes) {
    size_t off = size_t(static_cast<char*>(p) - base_), len = bytes;
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  size_t peak() const { return peak_; }

 private:
  char* base_;
  size_t bytes_;
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used_ = 0, peak_ = 0;
};

inline Arena*& active_arena() {
  static thread_local Arena* a = nullptr;
  return a;
}

struct ArenaScope {
  Arena* prev;
  explicit ArenaScope(Arena* a) : prev(active_arena()) { active_arena() = a; }
  ~ArenaScope() { active_arena() = prev; }
};

class Pool {
 public:
  static Pool& instance() {
    static Pool* p = new Pool();  // never destroyed: blocks may outlive static teardown
    return *p;
  }

  void* get(size_t bytes, hipStream_t s, size_t* got) {
    const size_t want = round(bytes);
    if (Arena* a = active_arena()) {
      *got = want;
      return a->get(want);
    }
    int dev = 0;
    KB_CHECK(hipGetDevice(&dev));
    Blk b{nullptr, 0, nullptr, 0, nullptr};
    bool found = false;
    {
      // take a block under the lock; wait for its last user only after
      // releasing the lock, so no thread blocks on the GPU while holding it
      std::lock_guard<std::mutex> lk(mu_);
      for (auto it = free_.lower_bound(want); it != free_.end() && it->first <= 2 * want; ++it) {
        if (it->second.dev != dev) continue;
        b = it->second;
        free_.erase(it);
        cached_ -= b.bytes;
        found = true;
        break;
      }
    }
    if (found) {
      if (b.ev) {
        // order the new user's stream after the last user's work on the
        // device; the host does not wait
        const hipError_t e1 = (b.stream != s) ? hipStreamWaitEvent(s, b.ev, 0) : hipSuccess;
        if (e1 != hipSuccess) {
          (void)hipGetLastError();
          (void)hipEventSynchronize(b.ev);
          (void)hipEventDestroy(b.ev);
          (void)hipFree(b.p);
          KB_CHECK(e1);
        }
        put_event(b.ev, dev);  // the wait (if any) is queued: the event may be recorded again
      }
      *got = b.bytes;
      return b.p;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      trim();
      e = hipMalloc(&p, want);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        throw OutOfMemory("hipMalloc of " + std::to_string(want) + " bytes failed");
      }
    }
    *got = want;
    return p;
  }

  void put(void* p, size_t bytes, hipStream_t s) {
    if (!p) return;
    if (Arena* a = active_arena()) {
      if (a->owns(p)) {
        a->put(p, bytes);
        return;
      }
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    Blk b{p, bytes, s, dev, get_event(dev)};
    if (!b.ev || hipEventRecord(b.ev, s) != hipSuccess) {
      // cannot order a later reuse: give the block back to the runtime
      (void)hipGetLastError();
      if (b.ev) (void)hipEventDestroy(b.ev);
      (void)hipStreamSynchronize(s);
      (void)hipFree(p);
      return;
    }
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace(bytes, b);
    cached_ += bytes;
  }

  // Releases every cached block (after the device has finished with them).
  void trim() {
    std::multimap<size_t, Blk> all;
    {
      std::lock_guard<std::mutex> lk(mu_);
      all.swap(free_);
      cached_ = 0;
    }
    for (auto& kv : all) {
      if (kv.second.ev) {
        (void)hipEventSynchronize(kv.second.ev);
        (void)hipEventDestroy(kv.second.ev);
      }
      (void)hipFree(kv.second.p);
    }
  }

  size_t cached_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return cached_;
  }

 private:
  struct Blk {
    void* p;
    size_t bytes;
    hipStream_t stream;
    int dev;
    hipEvent_t ev;
  };
  // Events of the current device are reused (a create and destroy per block
  // and job add up); nullptr when none can be created.
  hipEvent_t get_event(int dev) {
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = free_ev_.size(); i-- > 0;) {
        if (free_ev_[i].first != dev) continue;
        const hipEvent_t e = free_ev_[i].second;
        free_ev_.erase(free_ev_.begin() + long(i));
        return e;
      }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
  void put_event(hipEvent_t e, int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    free_ev_.emplace_back(dev, e);
  }
  static size_t round(size_t b) {
    if (b == 0) b = 1;
    const size_t g = (b >= (size_t(1) << 20) && !active_arena()) ? (size_t(1) << 20) : 256;
    return (b + g - 1) / g * g;
  }
  std::mutex mu_;
  std::multimap<size_t, Blk> free_;
  std::vector<std::pair<int, hipEvent_t>> free_ev_;
  size_t cached_ = 0;
};

// Small pinned host buffers for device-to-host readbacks, carved from one
// slab that lives until the process ends (per-handle pinned allocation and
// release would synchronise the whole device every time).
class PinnedSlots {
 public:
  static constexpr size_t kSlotWords = 64;
  static PinnedSlots& instance() {
    static PinnedSlots* p = new PinnedSlots();
    return *p;
  }
  uint64_t* acquire() {
    for (;;) {
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (!free_.empty()) {
          uint64_t* w = free_.back();
          free_.pop_back();
          return w;
        }
      }
      // allocate a new slab outside the lock
      void* slab = nullptr;
      const size_t n = 256;  // slots per slab
      if (hipHostMalloc(&slab, n * kSlotWords * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        throw OutOfMemory("hipHostMalloc of readback slots failed");
      }
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = 0; i < n; ++i) free_.push_back(static_cast<uint64_t*>(slab) + i * kSlotWords);
    }
  }
  void release(uint64_t* w) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(w);
  }

 private:
  std::mutex mu_;
  std::vector<uint64_t*> free_;
};

// Non-blocking streams of default priority for the resolvers of a graph
// handle, kept per device for the life of the process: creating and
// destroying two streams per job costs about 0.2 ms. A returned stream has
// been synchronised by its user.
class StreamPool {
 public:
  static StreamPool& instance() {
    static StreamPool* p = new StreamPool();  // never destroyed, like the streams
    return *p;
  }
  hipStream_t get() {
    int dev = 0;
    KB_CHECK(hipGetDevice(&dev));
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (size_t i = 0; i < free_.size(); ++i) {
        if (free_[i].first != dev) continue;
        const hipStream_t s = free_[i].second;
        free_.erase(free_.begin() + long(i));
        return s;
      }
    }
    hipStream_t s = nullptr;
    KB_CHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  void put(hipStream_t s, int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    free_.emplace_back(dev, s);
  }

 private:
  std::mutex mu_;
  std::vector<std::pair<int, hipStream_t>> free_;
};

// Stream on which the calling thread's library work runs; device buffers
// record it so the pool can order their reuse.
inline hipStream_t& current_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}

struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(current_stream()) { current_stream() = s; }
  ~StreamScope() { current_stream() = prev; }
};

}  // namespace kb
