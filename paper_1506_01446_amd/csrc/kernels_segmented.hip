// Segmented sort: many independent arrays described by a CSR offset table,
// sorted in one persistent launch.  Each segment runs the same flip network
// as the single-array sort, padded virtually to its own power of two.
//
// Workgroups pull segment indices from an atomic counter (in the library's
// per-device scratch), so the launch needs no host knowledge of the segment
// sizes.  A segment of up to 2^kSegTile keys is sorted in LDS; a longer one is
// sorted by its workgroup in place: every 2^kSegTile chunk is sorted in LDS,
// then for each further phase the long-stride steps run over the segment in
// global memory (it stays in L2) and the short-stride tail runs per chunk in
// LDS.  Within one workgroup, a barrier orders the global stores of one step
// before the loads of the next.
#include "device.hpp"
#include "launch.hpp"
#include "segmented.hpp"

namespace bitonic {

constexpr int kSegTile = 13;
constexpr int kSegThreads = 256;

__device__ __forceinline__ int ceil_log2_u32(uint32_t n) {
  return n <= 1 ? 0 : 32 - __clz(n - 1);
}

// One step of the network on LDS keys s[0, T): comparators of bit sb.
__device__ __forceinline__ void seg_lds_step(int32_t* s, uint32_t T, int sb, bool mirror) {
  for (uint32_t c = threadIdx.x; c < (T >> 1); c += kSegThreads) {
    const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
    const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
    const int32_t a = s[i], b = s[j];
    s[i] = min(a, b);
    s[j] = max(a, b);
  }
  __syncthreads();
}

// Load `valid` keys (pad to T with the sentinel) into LDS.
__device__ __forceinline__ void seg_lds_load(int32_t* s, const int32_t* src, uint32_t T,
                                             uint32_t valid, int32_t flip) {
  for (uint32_t i = threadIdx.x; i < T; i += kSegThreads)
    s[i] = i < valid ? (src[i] ^ flip) : kPad;
  __syncthreads();
}

__device__ __forceinline__ void seg_lds_store(const int32_t* s, int32_t* dst, uint32_t valid,
                                              int32_t flip) {
  for (uint32_t i = threadIdx.x; i < valid; i += kSegThreads) dst[i] = s[i] ^ flip;
  __syncthreads();
}

// One step over a whole segment in global memory (virtual padding at len).
__device__ __forceinline__ void seg_global_step(int32_t* a, uint32_t len, uint32_t half, int sb,
                                                bool mirror, int32_t flip) {
  for (uint32_t c = threadIdx.x; c < half; c += kSegThreads) {
    const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
    const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
    if (j >= len) continue;
    const int32_t x = a[i] ^ flip, y = a[j] ^ flip;
    if (x > y) {
      a[i] = y ^ flip;
      a[j] = x ^ flip;
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kSegThreads) void seg_persistent_kernel(
    int32_t* __restrict__ keys, const int64_t* __restrict__ offsets, int64_t nseg, int32_t flip,
    uint32_t* __restrict__ counter) {
  __shared__ int32_t s[1 << kSegTile];
  __shared__ int64_t item;
  for (;;) {
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(counter, 1u);
    __syncthreads();
    const int64_t seg = item;
    __syncthreads();
    if (seg >= nseg) break;
    const int64_t off = offsets[seg];
    const uint32_t len = (uint32_t)(offsets[seg + 1] - off);
    if (len <= 1) continue;
    int32_t* a = keys + off;
    const int m = ceil_log2_u32(len);
    if (m <= kSegTile) {
      const uint32_t T = 1u << m;
      seg_lds_load(s, a, T, len, flip);
      for (int p = 1; p <= m; ++p) {
        seg_lds_step(s, T, p - 1, true);
        for (int sb = p - 2; sb >= 0; --sb) seg_lds_step(s, T, sb, false);
      }
      seg_lds_store(s, a, len, flip);
      continue;
    }
    constexpr uint32_t T = 1u << kSegTile;
    const uint32_t nchunks = (len + T - 1) >> kSegTile;
    for (uint32_t ch = 0; ch < nchunks; ++ch) {
      const uint32_t c0 = ch << kSegTile;
      const uint32_t valid = min(len - c0, T);
      seg_lds_load(s, a + c0, T, valid, flip);
      for (int p = 1; p <= kSegTile; ++p) {
        seg_lds_step(s, T, p - 1, true);
        for (int sb = p - 2; sb >= 0; --sb) seg_lds_step(s, T, sb, false);
      }
      seg_lds_store(s, a + c0, valid, flip);
    }
    const uint32_t half = 1u << (m - 1);
    for (int p = kSegTile + 1; p <= m; ++p) {
      for (int sb = p - 1; sb >= kSegTile; --sb) seg_global_step(a, len, half, sb, sb == p - 1, flip);
      for (uint32_t ch = 0; ch < nchunks; ++ch) {
        const uint32_t c0 = ch << kSegTile;
        const uint32_t valid = min(len - c0, T);
        seg_lds_load(s, a + c0, T, valid, flip);
        for (int sb = kSegTile - 1; sb >= 0; --sb) seg_lds_step(s, T, sb, false);
        seg_lds_store(s, a + c0, valid, flip);
      }
    }
  }
}

__global__ void seg_reset_kernel(uint32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

void launch_segmented(int32_t* keys, const int64_t* offsets, int64_t nseg, int32_t flip,
                      uint32_t* counter, int grid, hipStream_t st) {
  seg_reset_kernel<<<1, 64, 0, st>>>(counter);
  seg_persistent_kernel<<<grid, kSegThreads, 0, st>>>(keys, offsets, nseg, flip, counter);
}

}  // namespace bitonic
