// Per-(device, stream) scratch buffers of the segmented sort (host code, no
// HIP: the allocator is a parameter, so the policy is tested on the CPU).
//
// A call on stream S takes S's buffer, growing it when the call needs more.
// Work already enqueued on S may still read the old buffer, so a replaced
// buffer is retired, never freed: it stays allocated until the process ends
// (growth by half again each time keeps the retired total below twice the
// largest buffer).  Nothing ever waits for the stream.  Calls on different
// streams use different buffers and may overlap; calls on one stream are
// ordered by it.
#pragma once

#include <stddef.h>

#include <mutex>
#include <vector>

namespace bitonic {

// Alloc: struct with `void* alloc(size_t bytes)` (nullptr on failure).
template <class Alloc>
class ScratchCache {
 public:
  explicit ScratchCache(Alloc a = Alloc{}) : alloc_(a) {}

  // The buffer of (dev, stream), at least `bytes` long; nullptr if the
  // allocation fails (the previous buffer then stays in place).
  void* get(int dev, const void* stream, size_t bytes) {
    std::lock_guard<std::mutex> lock(mu_);
    for (auto& s : slots_) {
      if (s.dev != dev || s.stream != stream) continue;
      if (s.bytes >= bytes) return s.ptr;
      const size_t want = bytes + bytes / 2;
      void* p = alloc_.alloc(want);
      if (!p) return nullptr;
      retired_.push_back(s.ptr);
      retired_bytes_ += s.bytes;
      s.ptr = p;
      s.bytes = want;
      return p;
    }
    const size_t want = bytes < kMinBytes ? kMinBytes : bytes;
    void* p = alloc_.alloc(want);
    if (!p) return nullptr;
    slots_.push_back({dev, stream, p, want});
    return p;
  }

  size_t retired_count() const { return retired_.size(); }
  size_t retired_bytes() const { return retired_bytes_; }
  size_t live_bytes() const {
    size_t b = 0;
    for (const auto& s : slots_) b += s.bytes;
    return b;
  }
  Alloc& allocator() { return alloc_; }

  static constexpr size_t kMinBytes = size_t(1) << 20;

 private:
  struct Slot {
    int dev;
    const void* stream;
    void* ptr;
    size_t bytes;
  };
  Alloc alloc_;
  std::mutex mu_;
  std::vector<Slot> slots_;
  std::vector<void*> retired_;
  size_t retired_bytes_ = 0;
};

}  // namespace bitonic
