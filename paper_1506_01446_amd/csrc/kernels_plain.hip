// Kernels of the single-array sort.
//
//  (tile_kernel, tile_loop_kernel  the tile sort and merge: tile_kernels.hpp,
//                         instantiated here for 2^11..2^13-key tiles)
//  (global_pass_kernel    the fused long-stride passes: kernels_pass.hip)
//  lds_network_kernel     the same network steps with one compare-exchange per
//                         thread per step in LDS (section 4.1 as written)
//  step_kernel            one step, one compare-exchange per thread, in global
//                         memory (the basic scheme of section 3.3)
//
// All kernels sort ascending in the codec domain (see Codec) and treat indices
// >= n as absent INT32_MAX sentinels.  The tile and pass kernels of a sort
// apply the codec only where the sort's data enters and leaves them (CX, see
// KeyIO); the LDS-network and step kernels apply it at every access.
#include "device.hpp"
#include "launch.hpp"
#include "tile_kernels.hpp"

namespace bitonic {

// One step in LDS per iteration: comparator c of the step (lower index i has
// bit sb clear) meets i | 2^sb, or its mirror i ^ (2^(sb+1) - 1).
__device__ __forceinline__ void lds_step(int32_t* s, uint32_t T, int sb, bool mirror) {
  for (uint32_t c = threadIdx.x; c < (T >> 1); c += blockDim.x) {
    const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
    const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
    const int32_t a = s[i], b = s[j];
    s[i] = min(a, b);
    s[j] = max(a, b);
  }
  __syncthreads();
}

// Tile of 2^L keys (L <= 13) in LDS.  tail == 0: phases p_first..p_last
// (each a mirror step and half-cleaners); tail != 0: strides 2^(L-1)..1.
__global__ __launch_bounds__(1024) void lds_network_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                           int L, int p_first, int p_last,
                                                           int tail, Codec cd) {
  extern __shared__ int32_t s[];
  const uint32_t T = 1u << L;
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < T ? left : T;
  for (uint32_t i = threadIdx.x; i < T; i += blockDim.x)
    s[i] = i < valid ? cd.enc(keys[t0 + i]) : kPad;
  __syncthreads();
  if (tail) {
    for (int sb = L - 1; sb >= 0; --sb) lds_step(s, T, sb, false);
  } else {
    for (int p = p_first; p <= p_last; ++p) {
      lds_step(s, T, p - 1, true);
      for (int sb = p - 2; sb >= 0; --sb) lds_step(s, T, sb, false);
    }
  }
  for (uint32_t i = threadIdx.x; i < valid; i += blockDim.x) keys[t0 + i] = cd.dec(s[i]);
}

// One step of the network in global memory, one comparator per thread.
__global__ __launch_bounds__(256) void step_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                   uint32_t half, int sb, int mirror,
                                                   Codec cd) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= half) return;
  const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
  const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
  if (j >= n) return;
  const int32_t a = cd.enc(keys[i]), b = cd.enc(keys[j]);
  if (a > b) {
    keys[i] = cd.dec(b);
    keys[j] = cd.dec(a);
  }
}

// ---------------------------------------------------------------------------
// launchers

bool tile_log2_supported(int L) { return L >= kTileMinLog2 && L <= kTileMaxLog2; }

void launch_tile(int L, int kind, int32_t* keys, uint32_t n, Codec cd, int cx,
                 uint32_t max_blocks, hipStream_t st) {
  switch (L) {
    case 11: launch_tile_L<11>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 12: launch_tile_L<12>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 13: launch_tile_L<13>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 14: launch_tile_14(kind, keys, n, cd, cx, max_blocks, st); break;
    case 15: launch_tile_15(kind, keys, n, cd, cx, max_blocks, st); break;
    default: break;
  }
}

void launch_tile_scalar(int kind, int32_t* keys, uint32_t n, Codec cd, int cx, hipStream_t st) {
  constexpr int L = kScalarTileLog2;
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (codec_is_identity(cd)) cx = CX_NONE;
  if (kind == 0) {  // the scalar-I/O sort with lane steps (program kind 6)
    if (cx == CX_NONE)
      tile_kernel<L, kTileRegLog, 6, CX_NONE><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else if (cx == CX_ENC)
      tile_kernel<L, kTileRegLog, 6, CX_ENC><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else
      tile_kernel<L, kTileRegLog, 6, CX_BOTH><<<ntiles, NT, 0, st>>>(keys, n, cd);
  } else if (cx == CX_NONE) {
    tile_kernel<L, kTileRegLog, 3, CX_NONE><<<ntiles, NT, 0, st>>>(keys, n, cd);
  } else {
    tile_kernel<L, kTileRegLog, 3, CX_DEC><<<ntiles, NT, 0, st>>>(keys, n, cd);
  }
}

void launch_lds_network(int L, int p_first, int p_last, bool tail, int32_t* keys, uint32_t n,
                        Codec cd, hipStream_t st) {
  const uint32_t T = 1u << L;
  const uint32_t blocks = (uint32_t)(((uint64_t)n + T - 1) >> L);
  uint32_t threads = T / 2;
  if (threads > 1024) threads = 1024;
  if (threads < 64) threads = 64;
  lds_network_kernel<<<blocks, threads, T * sizeof(int32_t), st>>>(keys, n, L, p_first, p_last,
                                                                   tail ? 1 : 0, cd);
}

void launch_step(int sb, bool mirror, int32_t* keys, uint32_t n, uint32_t N, Codec cd,
                 hipStream_t st) {
  const uint32_t half = N >> 1;
  const uint32_t blocks = (half + 255) / 256;
  step_kernel<<<blocks, 256, 0, st>>>(keys, n, half, sb, mirror ? 1 : 0, cd);
}

}  // namespace bitonic
