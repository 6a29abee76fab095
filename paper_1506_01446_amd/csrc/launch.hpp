// Host-side launchers of the library's kernels (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.hpp"

namespace bitonic {

constexpr int kTileRegLogPlain = 5;  // 32 keys per thread in the tile kernels
constexpr int kFuseMaxFourColumn = 5;  // wider aligned passes take the one-column kernel
constexpr int kTileMinLog2 = 11;
constexpr int kTileMaxLog2 = 15;
constexpr int kFuseMaxColumn = 8;  // steps one thread's registers hold (one column)
constexpr int kFuseMax = 10;       // with a column split over lanes (lane passes)
constexpr int kFuseMaxRagged = 7;  // n not a power of two (see enqueue_plain)
constexpr int kLdsNetworkMaxLog2 = 13;

bool tile_log2_supported(int L);

// Tile sort (kind 0: phases 1..L; kind 4: the same with its steps on lane
// bits as cross-lane steps), tile merge (kind 1: strides 2^(L-1)..1) or
// tile phase (kind 5, L >= 12: phase L, for tiles whose halves are each
// ascending) over every 2^L tile of keys[0, n).  Merges and phases run at
// most max_blocks workgroups (0 = one per tile), each looping over its
// tiles.  cx (CX_*): whether loads encode and stores decode; a tile sort
// takes CX_ENC or CX_BOTH, a merge or phase CX_NONE or CX_DEC.
void launch_tile(int L, int kind, int32_t* keys, uint32_t n, Codec cd, int cx,
                 uint32_t max_blocks, hipStream_t st);

// Arrays that do not start on a 16-byte boundary: tile sort (kind 0) or merge
// (kind 1) of 2^kScalarTileLog2-key tiles whose global accesses put lanes on
// consecutive keys (4-byte alignment suffices).  cx as for launch_tile.
constexpr int kScalarTileLog2 = 13;
void launch_tile_scalar(int kind, int32_t* keys, uint32_t n, Codec cd, int cx, hipStream_t st);

// f fused steps on bits q+f-1 .. q (the first one the mirror step if
// `mirror`) on keys already in the sorting domain.  Requires q >= 8,
// q + f <= 31, 1 <= f <= kFuseMaxColumn (f <= 5: four columns per thread;
// 6..8: one column).
void launch_global_pass(int f, bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st);

// The one-column passes: behind launch_global_pass for f = 6 .. kFuseMaxColumn,
// and for every f (1 .. kFuseMaxColumn) in the plan for unaligned arrays.
void launch_column_pass_i32(int f, bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st);

// Lane passes (column_lanes_pass_kernel): f = fr + g steps, each column split
// over 2^g lanes of 2^fr keys; (fr, g) in {7, 8} x {1, 2}; any n, the last
// block padded virtually (lane_pass_fits).  fr = -7, -8: the column over the
// four waves of a workgroup instead (column_waves_pass_kernel, f = 9, 10),
// whole blocks only: n a multiple of 2^(q+f) (wave_pass_fits).  Both need
// q + f <= 30.  False (nothing launched) for any other shape.
constexpr bool lane_pass_fits(uint32_t n, int q, int f) {
  return q + f <= 30 && q >= 8 && n != 0;
}
constexpr bool wave_pass_fits(uint32_t n, int q, int f) {
  return lane_pass_fits(n, q, f) && (n & ((uint32_t(1) << (q + f)) - 1u)) == 0;
}
bool launch_column_lanes_pass(int f, int fr, bool mirror, int32_t* keys, uint32_t n, int q,
                              hipStream_t st);

// LDS network on 2^L tiles (L <= kLdsNetworkMaxLog2).
void launch_lds_network(int L, int p_first, int p_last, bool tail, int32_t* keys, uint32_t n,
                        Codec cd, hipStream_t st);

// One step (bit sb; mirror or half-cleaner) over keys[0, n) padded to N.
void launch_step(int sb, bool mirror, int32_t* keys, uint32_t n, uint32_t N, Codec cd,
                 hipStream_t st);

// Sort of 8-byte elements (kernels_wide.hip): 2^kWideRegLog elements per
// thread in the tile kernels, tiles of 2^kWideTileMinLog2 .. 2^kWideTileMaxLog2
// elements, up to kWideFuseMax steps per pass.
constexpr int kWideRegLog = 4;
constexpr int kWideTileMinLog2 = 11;
constexpr int kWideTileMaxLog2 = 13;
constexpr int kWideFuseMaxColumn = 6;  // steps one thread's registers hold
constexpr int kWideFuseMax = 8;        // with a column split over lanes (lane passes)
constexpr int kWideLaneRegLog = 6;     // elements per lane of a lane pass, log2

// Lane passes of an 8-byte sort (f = 7, 8): whole 2^(q+f) blocks, and lane
// byte offsets below 2^32 for 8-byte units (so for either storage).
constexpr bool wide_lanes_fit(uint32_t n, int q, int f) {
  return q + f <= 29 && q >= 8 && n != 0 && (n & ((uint32_t(1) << (q + f)) - 1u)) == 0;
}

// Tile sort (kind 0) or merge (kind 1) over the 2^L-element tiles of an
// 8-byte sort: int64 keys at keys64 (values == nullptr), or pairs of 4-byte
// keys at keys32 and int32 values.  cx as for launch_tile.
void launch_wide_tile(int L, int kind, int64_t* keys64, int32_t* keys32, int32_t* values,
                      uint32_t n, Codec64 cd, int cx, hipStream_t st);

// Phase L (program kind 7: the mirror step, then strides 2^(L-2)..1) over
// the 2^L-element tiles of an 8-byte sort whose halves are each ascending,
// L = kWideTileMinLog2 + 1 .. kWideTileMaxLog2 + 1: phase t+1 after the tile
// sort of 2^t-element tiles in one launch.  cx CX_NONE or CX_DEC.
void launch_wide_phase(int L, int64_t* keys64, int32_t* keys32, int32_t* values, uint32_t n,
                       Codec64 cd, int cx, hipStream_t st);

// f fused steps on bits q+f-1 .. q of an 8-byte sort, on mapped elements.
// Requires q + f <= 31, 1 <= f <= kWideFuseMax, and wide_lanes_fit for
// f > kWideFuseMaxColumn.
void launch_wide_pass(int f, bool mirror, int64_t* keys64, int32_t* keys32, int32_t* values,
                      uint32_t n, int q, hipStream_t st);

// Width of the lane byte offsets a one-column pass forms for rows of 2^q
// elements of `unit` bytes: 32 bits while 2^q * unit <= 2^32, else 64.  Sorts
// hold n <= 2^31 elements and q + f <= 31, so only one-step passes of 8-byte
// elements at q = 30 (phase 31) need 64; the launcher instantiates the
// 64-bit form for exactly those (column_pass.hpp).
constexpr int pass_offset_bits(uint32_t unit, int q) {
  return ((uint64_t)unit << q) <= (uint64_t(1) << 32) ? 32 : 64;
}
constexpr int column_pass_offset_bits(uint32_t unit, int f, int q) {
  return (f == 1 && unit > 4) ? pass_offset_bits(unit, q) : 32;
}

// Input generator.
void launch_keygen(int32_t* out, uint64_t n, uint64_t seed, uint64_t start, hipStream_t st);

}  // namespace bitonic
