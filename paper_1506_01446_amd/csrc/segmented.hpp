// Segmented sort: scratch layout and launchers (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.hpp"

namespace bitonic {

constexpr int kTileRegLogSeg = 5;  // 32 keys per thread
constexpr int kSegSmallMaxLog2 = 13;  // segments of up to 2^13 keys are "small"
// Tiles of the big segments: 2^14 4-byte keys (the single-array sort's tile,
// 67.6 KB of LDS, two workgroups per CU), 2^13 8-byte elements (regrouped
// through half the LDS, 34 KB, four per CU).
constexpr int kSegTileLog32 = 14;
constexpr int kSegTileLog64 = 13;
constexpr int kSmallClasses = 9;   // classes 13, 12, ..., 6 and "<= 5"
constexpr int kSegFuseMax = 5;  // most steps per big-segment pass

// Written by the prep kernel, read by the others (device memory).
struct SegMeta {
  uint32_t small_counter;  // work queue of the small-segment kernel
  uint32_t small_items;    // work items in all
  uint32_t nbig;           // segments of class > 13
  int32_t max_class;       // largest class present (0 if no big segment)
  uint32_t small_start[kSmallClasses];  // first id of each small class bucket
  uint32_t small_count[kSmallClasses];
  uint32_t item_prefix[kSmallClasses + 1];
  uint32_t big_ge[33];     // number of big segments of class >= c
  int32_t invalid;         // set by the validation kernel: the table is refused
};
static_assert(sizeof(SegMeta) <= 1024, "the segment meta block takes the scratch's first KiB");

// Errors the validation kernel finds in a segment table (first one wins).
enum SegTableError : int32_t {
  kSegTableOk = 0,
  kSegTableDecreasing = 1,  // offsets[s + 1] < offsets[s]
  kSegTableTooLong = 2,     // a segment of 2^31 keys or more
  kSegTableOverBound = 3,   // a segment longer than the caller's bound
  kSegTableNegative = 4     // offsets[0] < 0
};

// Pointers into the scratch buffer of one segmented call (device memory).
struct SegScratch {
  SegMeta* meta;
  uint32_t* small_ids;   // nseg entries, bucketed by class, class 13 first
  uint32_t* big_ids;     // nseg entries, largest class first
  uint64_t* big_keys;    // nseg + 1: exclusive prefix of padded sizes
  uint64_t* big_tiles;   // nseg + 1: exclusive prefix of big-segment tiles
};

constexpr size_t seg_scratch_bytes(int64_t nseg) {
  const size_t n = (size_t)nseg + 1;
  return 1024 + 2 * ((4 * n + 255) & ~size_t(255)) + 2 * ((8 * n + 255) & ~size_t(255));
}

// The allocation-free entry point's scratch (noalloc.hip): a file-scope
// device array holding the segment table of up to kNoAllocMaxSegments
// segments (seg_scratch_bytes(2^18 - 1) = 6 MiB + 1 KiB).
constexpr int64_t kNoAllocMaxSegments = (int64_t(1) << 18) - 1;
constexpr size_t kNoAllocScratchBytes = 1024 + (size_t(24) << 18);

// Device address of that array on device `dev` (the current device), taken
// on the first call per device; 0 on success, -1 on a HIP error.
int noalloc_scratch(int dev, void** out);

inline SegScratch seg_scratch_carve(void* base, int64_t nseg) {
  const size_t n = (size_t)nseg + 1;
  char* p = static_cast<char*>(base);
  SegScratch s;
  s.meta = reinterpret_cast<SegMeta*>(p);
  p += 1024;
  s.small_ids = reinterpret_cast<uint32_t*>(p);
  p += (4 * n + 255) & ~size_t(255);
  s.big_ids = reinterpret_cast<uint32_t*>(p);
  p += (4 * n + 255) & ~size_t(255);
  s.big_keys = reinterpret_cast<uint64_t*>(p);
  p += (8 * n + 255) & ~size_t(255);
  s.big_tiles = reinterpret_cast<uint64_t*>(p);
  return s;
}

// The data of one segmented sort: 4-byte keys (keys, codec cd), (key,
// value) pairs moving as 8-byte elements (keys and values, codec cd64), or
// 8-byte keys (keys64, codec cd64).
struct SegData {
  int32_t* keys;
  int32_t* values;
  int64_t* keys64;
  Codec cd;
  Codec64 cd64;
};

// One launch of the sequence: the small-segment kernel, a big-segment tile
// sort or merge of the segments of class >= cls, or a pass of f steps on
// bits q+f-1 .. q of them.
struct SegLaunch {
  enum : int { kSmall = 0, kTileSort = 1, kTileMerge = 2, kPass = 3, kPhase = 4 };
  int what;
  int f;
  bool mirror;
  int cls;
  int q;
  int grid;
};

// Per storage type (kernels_seg32.hip, kernels_segpairs.hip, kernels_seg64.hip).
void seg_run_keys32(const SegData& d, const SegLaunch& l, const int64_t* offsets,
                    const SegScratch& sc, hipStream_t st);
void seg_run_pairs(const SegData& d, const SegLaunch& l, const int64_t* offsets,
                   const SegScratch& sc, hipStream_t st);
void seg_run_keys64(const SegData& d, const SegLaunch& l, const int64_t* offsets,
                    const SegScratch& sc, hipStream_t st);

// tile_log: log2 of the big segments' tile (kSegTileLog32 or kSegTileLog64).
// validated: a validation kernel ran first (launch_seg_validate); an invalid
// table then classifies as empty, so no later kernel touches the keys.
void launch_seg_prep(const int64_t* offsets, int64_t nseg, const SegScratch& sc, int tile_log,
                     bool validated, hipStream_t st);

// Checks offsets[0 .. nseg] (nondecreasing, offsets[0] >= 0, every segment
// below 2^31 keys and at most `bound` keys) on the device; records the first
// error of the call in sc.meta->invalid and in the device's error word
// (seg_validation_error) if that is still clear.
void launch_seg_validate(const int64_t* offsets, int64_t nseg, int64_t bound, const SegScratch& sc,
                         hipStream_t st);

// Reads (and then clears) the current device's error word: the first error
// (SegTableError) any validated call recorded since the last read.  Blocks
// until the device is idle.  0 on success, -1 on a HIP error.
int seg_validation_error(int32_t* code);
void launch_seg_small(const SegData& d, const int64_t* offsets, const SegScratch& sc, int grid,
                      hipStream_t st);
// Tile sort (merge == false) or tile merge of the big segments of class >= cls_min.
void launch_seg_tiles(bool merge, const SegData& d, const int64_t* offsets, const SegScratch& sc,
                      int cls_min, int grid, hipStream_t st);
// f fused steps on bits q+f-1 .. q of the big segments of class >= cls.
void launch_seg_pass(int f, bool mirror, const SegData& d, const int64_t* offsets,
                     const SegScratch& sc, int cls, int q, int grid, hipStream_t st);
// Phase T + 1 of the big segments of that class or above (T the big
// segments' tile log2): one launch instead of a one-step pass and a tile
// merge.
void launch_seg_phase(const SegData& d, const int64_t* offsets, const SegScratch& sc, int grid,
                      hipStream_t st);

}  // namespace bitonic
