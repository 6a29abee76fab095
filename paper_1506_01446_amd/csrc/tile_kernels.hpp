// Tile kernels of the single-array sort of 4-byte keys (templates; each
// tile size is instantiated in a file of its own so that they compile in
// parallel: kernels_plain.hip for 2^11..2^13, kernels_tile14.hip,
// kernels_tile15.hip).
//
//  tile_kernel<L, r, 0, CX>       phases 1..L of the network on every 2^L
//                                 tile, keys in registers, regrouped through
//                                 LDS (the paper's shared-memory
//                                 optimization, section 4.1, with the
//                                 register blocking of section 4.2 inside
//                                 the tile)
//  tile_kernel<L, r, 4, CX>       the same with every step on an index bit
//                                 that a wave holds across its lanes done by
//                                 cross-lane compare-exchanges (DPP, permlane
//                                 swaps) instead of LDS regroups
//  tile_kernel<L, r, 1, CX>       the last L steps (strides 2^(L-1)..1) of a
//                                 phase longer than the tile, on every tile
//  tile_kernel<L, r, 5, CX>       phase L (mirror step, then strides
//                                 2^(L-2)..1) on every tile: phase t+1 of a
//                                 sort with 2^t-key tiles in one launch
//  tile_loop_kernel<L, r, K, CX>  the same (K = 1, 5), each workgroup
//                                 looping over several tiles
#pragma once

#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

// One tile per workgroup.
template <int L, int RL, int KIND, int CX>
__global__ __launch_bounds__(1 << (L - RL)) void tile_kernel(int32_t* __restrict__ keys,
                                                             uint32_t n, Codec codec) {
  using PR = Prog<L, RL, KIND>;
  __shared__ int32_t lds[PR::LDSW];
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < (uint32_t)PR::T ? left : (uint32_t)PR::T;
  tile_program<PR>(keys + t0, valid, KeyIO<CX>{codec}, lds, threadIdx.x);
}

// The full tiles blockIdx.x, blockIdx.x + gridDim.x, ... of keys[0, n), then
// the partial last tile (if any) on one block.  The keys of a block's next
// tile are loaded into a second register set before the current tile's steps
// run, so that those loads are in flight while the tile is processed and
// stored (the workgroup barriers wait for LDS traffic only).  The next tile is
// read through a buffer resource that is empty when there is no next tile, so
// every iteration issues the same loads: with a load in a branch the
// compiler would wait for all loads at the join, the prefetch included.  The
// thread id is passed through an empty asm statement every iteration so that
// the compiler recomputes the loop-invariant LDS and global offsets instead
// of keeping all of them live in registers.
template <int L, int RL, int KIND, int CX>
__global__ __launch_bounds__(1 << (L - RL)) void tile_loop_kernel(int32_t* __restrict__ keys,
                                                                  uint32_t n, Codec codec) {
  using PR = Prog<L, RL, KIND>;
  constexpr int LAST = PR::value.ngroups - 1;
  static_assert(layout_is_vector4(PR::value.g[LAST]), "16-byte store layout expected");
  const KeyIO<CX> cd{codec};
  __shared__ int32_t lds[PR::LDSW];
  const uint32_t nfull = n >> L;
  auto rsrc_of = [&](uint32_t tile) {
    return tile_rsrc(keys + ((size_t)tile << L), tile < nfull ? (uint32_t)PR::T * 4u : 0u);
  };
  uint32_t tile = blockIdx.x;
  int32_t x[PR::R];
  load_tile_rsrc<PR, 0>(x, rsrc_of(tile), cd, threadIdx.x);
  // Wait for the first tile here, so that at the loop head only the
  // previous iteration's prefetch has to be waited for, not its stores.
#pragma unroll
  for (int j = 0; j < PR::R; ++j) asm volatile("" : "+v"(x[j]));
  for (; tile < nfull; tile += gridDim.x) {
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    int32_t y[PR::R];
    load_tile_rsrc<PR, 0>(y, rsrc_of(tile + gridDim.x), cd, tid);
    run_from<PR, 0>(x, lds, tid);
    store_tile<PR, LAST>(x, keys + ((size_t)tile << L), (uint32_t)PR::T, cd, tid);
    static_for<0, PR::R>([&](auto J) { x[J] = y[J]; });
  }
  const uint32_t rest = n & (uint32_t)(PR::T - 1);
  if (rest != 0 && blockIdx.x == nfull % gridDim.x)
    tile_program<PR>(keys + ((size_t)nfull << L), rest, cd, lds, threadIdx.x);
}

constexpr int kTileRegLog = kTileRegLogPlain;

template <int L, int KIND, int CX>
inline void launch_merge_LC(int32_t* keys, uint32_t n, Codec cd, uint32_t max_blocks,
                            hipStream_t st) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (max_blocks == 0 || max_blocks >= ntiles)
    tile_kernel<L, kTileRegLog, KIND, CX><<<ntiles, NT, 0, st>>>(keys, n, cd);
  else
    tile_loop_kernel<L, kTileRegLog, KIND, CX><<<max_blocks, NT, 0, st>>>(keys, n, cd);
}

// Instantiated codec modes: a tile sort is a sort's first kernel (CX_ENC, or
// CX_BOTH when it is the only one), a merge is never its first (CX_DEC for the
// last); CX_NONE serves the identity codec and the kernels in between.
template <int L>
inline void launch_tile_L(int kind, int32_t* keys, uint32_t n, Codec cd, int cx,
                          uint32_t max_blocks, hipStream_t st) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (codec_is_identity(cd)) cx = CX_NONE;
  if (kind == 0) {
    if (cx == CX_NONE)
      tile_kernel<L, kTileRegLog, 0, CX_NONE><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else if (cx == CX_ENC)
      tile_kernel<L, kTileRegLog, 0, CX_ENC><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else
      tile_kernel<L, kTileRegLog, 0, CX_BOTH><<<ntiles, NT, 0, st>>>(keys, n, cd);
  } else if (kind == 4) {  // the sort with lane steps (program kind 4)
    if (cx == CX_NONE)
      tile_kernel<L, kTileRegLog, 4, CX_NONE><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else if (cx == CX_ENC)
      tile_kernel<L, kTileRegLog, 4, CX_ENC><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else
      tile_kernel<L, kTileRegLog, 4, CX_BOTH><<<ntiles, NT, 0, st>>>(keys, n, cd);
  } else if (kind == 5) {  // one whole phase (program kind 5), 2^12..2^15 tiles
    if constexpr (L >= 12) {
      if (cx == CX_NONE)
        launch_merge_LC<L, 5, CX_NONE>(keys, n, cd, max_blocks, st);
      else
        launch_merge_LC<L, 5, CX_DEC>(keys, n, cd, max_blocks, st);
    }
  } else if (cx == CX_NONE) {
    launch_merge_LC<L, 1, CX_NONE>(keys, n, cd, max_blocks, st);
  } else {
    launch_merge_LC<L, 1, CX_DEC>(keys, n, cd, max_blocks, st);
  }
}

// Instantiated in kernels_tile14.hip and kernels_tile15.hip.
void launch_tile_14(int kind, int32_t* keys, uint32_t n, Codec cd, int cx, uint32_t max_blocks,
                    hipStream_t st);
void launch_tile_15(int kind, int32_t* keys, uint32_t n, Codec cd, int cx, uint32_t max_blocks,
                    hipStream_t st);

}  // namespace bitonic
