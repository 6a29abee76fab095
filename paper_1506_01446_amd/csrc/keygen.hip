// Input generator on the device (not part of the sorting method): the
// counter-based SplitMix64 stream of Steele, Lea and Flood (2014).  Word i of
// stream `seed` is mix(seed + (i + 1) * 0x9E3779B97F4A7C15); a key is its
// high 32 bits read as a signed int32.
#include "launch.hpp"

namespace bitonic {

__device__ __forceinline__ uint64_t splitmix64_word(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void keygen_kernel(int32_t* __restrict__ out, uint64_t n,
                                                     uint64_t seed, uint64_t start) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n; i += stride)
    out[i] = (int32_t)(uint32_t)(splitmix64_word(seed, start + i) >> 32);
}

void launch_keygen(int32_t* out, uint64_t n, uint64_t seed, uint64_t start, hipStream_t st) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks == 0) return;
  keygen_kernel<<<(uint32_t)blocks, 256, 0, st>>>(out, n, seed, start);
}

}  // namespace bitonic
