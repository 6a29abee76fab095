// The scratch of the allocation-free segmented sort
// (bitonic_sort_segmented_noalloc_i32): one file-scope device array of
// kNoAllocScratchBytes, which every GPU the library runs on holds until the
// process ends.  Its device address is taken once per device, with that
// device current, through hipGetSymbolAddress; host code uses only that
// address (in host code the array's own name is a host-side stand-in, not a
// device address).
#include <atomic>

#include "launch.hpp"
#include "segmented.hpp"

namespace bitonic {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static_assert(seg_scratch_bytes(kNoAllocMaxSegments) <= kNoAllocScratchBytes,
              "scratch too small for the largest segment table");

namespace {
constexpr int kMaxDev = 64;
std::atomic<void*> g_ptr[kMaxDev];
}  // namespace

int noalloc_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDev) return -1;
  void* p = g_ptr[dev].load(std::memory_order_acquire);
  if (!p) {
    // first call on this device (which is current): take the array's device
    // address; concurrent first calls store the same address
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    g_ptr[dev].store(p, std::memory_order_release);
  }
  *out = p;
  return 0;
}

}  // namespace bitonic
