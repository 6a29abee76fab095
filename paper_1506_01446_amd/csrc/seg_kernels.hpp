// Kernel templates of the segmented sort (see kernels_segmented.hip), over a
// storage type ST (column_pass.hpp): Keys32, Keys64 or Pairs.  Each storage
// is instantiated in a file of its own (kernels_seg32.hip,
// kernels_segpairs.hip, kernels_seg64.hip) so that they compile in parallel.
#pragma once

#include <type_traits>

#include "column_pass.hpp"
#include "device.hpp"
#include "launch.hpp"
#include "segmented.hpp"
#include "split_regroup.hpp"

namespace bitonic {

constexpr int kSegThreads = 256;

__device__ __forceinline__ int ceil_log2_u64(uint64_t n) {
  return n <= 1 ? 0 : 64 - __clzll(n - 1);
}

// Small classes 13, 12, ..., 6, and "<= 5" (index 8): segments per item.
__device__ __forceinline__ int small_class_of_index(int i) { return 13 - i; }  // 5 for i == 8
__device__ __forceinline__ uint32_t small_per_item(int cls) {
  return cls <= 5 ? 256u : (256u >> (cls - 5));
}

// Storage ST of a segmented sort: Keys32 (4-byte keys, Codec) or Pairs
// (key, value pairs as 8-byte elements, Codec64); every kernel maps keys into
// the sorting domain as it loads them and back as it stores them.
//
// One tile of a storage in a scalar-I/O program (KIND 2 or 3), `valid` of its
// elements real.  4-byte keys take the single-array sort's tile program.
//
// SPLIT (8-byte elements only): lds is an array of PR::LDSW 4-byte words and
// the regroups move high and low words in turn (run_from_split).
template <class PR, bool SPLIT = false, class ST, class CD>
__device__ __forceinline__ void seg_tile_program(ST tile, uint32_t valid, CD cd,
                                                 typename ST::E* lds, uint32_t tid) {
  if constexpr (std::is_same_v<ST, Keys32>) {
    tile_program<PR>(tile.k, valid, cd, lds, tid);
  } else {
    using E = typename ST::E;
    constexpr int LAST = PR::value.ngroups - 1;
    const bool full = valid >= (uint32_t)PR::T;
    E x[PR::R];
    {
      constexpr Group gr = PR::value.g[0];
      const uint32_t base = deposit<free_mask(gr, PR::L)>(tid);
      if (full) {
        static_for<0, PR::R>([&](auto J) { x[J] = cd.enc(tile.get(slot_index<PR, 0, J>(base))); });
      } else {
        static_for<0, PR::R>([&](auto J) {
          const uint32_t i = slot_index<PR, 0, J>(base);
          x[J] = i < valid ? cd.enc(tile.get(i)) : ST::kPadE;
        });
      }
    }
    if constexpr (SPLIT)
      run_from_split<PR, 0>(x, reinterpret_cast<uint32_t*>(lds), tid);
    else
      run_from<PR, 0>(x, lds, tid);
    {
      if constexpr (PR::LEAN) asm volatile("" : "+v"(tid));
      constexpr Group gr = PR::value.g[LAST];
      const uint32_t base = deposit<free_mask(gr, PR::L)>(tid);
      if (full) {
        static_for<0, PR::R>([&](auto J) { tile.put(slot_index<PR, LAST, J>(base), cd.dec(x[J])); });
      } else {
        static_for<0, PR::R>([&](auto J) {
          const uint32_t i = slot_index<PR, LAST, J>(base);
          if (i < valid) tile.put(i, cd.dec(x[J]));
        });
      }
    }
  }
}

// The scalar-I/O tile-sort program of a storage: with lane steps (kind 6)
// for 4-byte keys, without (kind 2) for 8-byte elements.
template <class ST>
constexpr int seg_sort_kind() {
  return sizeof(typename ST::E) == 4 ? 6 : 2;
}

// ---------------------------------------------------------------------------
// small segments

constexpr uint32_t kSmallLdsWords = (kSegThreads << kTileRegLogSeg) / 32 * 33;

// Not inlined: each class's program keeps its own register allocation
// instead of the kernel carrying the union of all of them.
template <int L, class ST, class CD>
__device__ __attribute__((noinline)) void seg_small_item(ST keys,
                                               const int64_t* __restrict__ offsets,
                                               const uint32_t* __restrict__ ids, uint32_t first,
                                               uint32_t count, CD cd, typename ST::E* lds) {
  using PR = Prog<L, kTileRegLogSeg, seg_sort_kind<ST>()>;
  constexpr uint32_t NT = PR::NT;
  static_assert((kSegThreads / NT) * PR::LDSW <= kSmallLdsWords, "padded tiles exceed LDS");
  const uint32_t grp = threadIdx.x / NT;
  const uint32_t ltid = threadIdx.x % NT;
  ST p = keys;
  uint32_t len = 0;
  if (grp < count) {
    const uint32_t s = ids[first + grp];
    const int64_t off = offsets[s];
    p = keys.at(off);
    len = (uint32_t)(offsets[s + 1] - off);
  }
  seg_tile_program<PR>(p, len, cd, lds + grp * PR::LDSW, ltid);
}

template <class ST, class CD>
__global__ __launch_bounds__(kSegThreads) void seg_small_kernel(
    ST keys, const int64_t* __restrict__ offsets, SegMeta* __restrict__ meta,
    const uint32_t* __restrict__ small_ids, CD cd) {
  // room for 256 / 2^(m-5) padded tiles of 2^m elements, for every class m
  __shared__ typename ST::E lds[kSmallLdsWords];
  __shared__ uint32_t item_s;
  const uint32_t total = meta->small_items;
  for (;;) {
    if (threadIdx.x == 0) item_s = atomicAdd(&meta->small_counter, 1u);
    __syncthreads();
    const uint32_t item = item_s;
    __syncthreads();
    if (item >= total) break;
    int ci = 0;
    while (ci + 1 < kSmallClasses && meta->item_prefix[ci + 1] <= item) ++ci;
    const int cls = small_class_of_index(ci);
    const uint32_t per = small_per_item(cls);
    const uint32_t k = item - meta->item_prefix[ci];
    const uint32_t first = meta->small_start[ci] + k * per;
    const uint32_t left = meta->small_count[ci] - k * per;
    const uint32_t count = left < per ? left : per;
    switch (cls) {
      case 13: seg_small_item<13>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 12: seg_small_item<12>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 11: seg_small_item<11>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 10: seg_small_item<10>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 9: seg_small_item<9>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 8: seg_small_item<8>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 7: seg_small_item<7>(keys, offsets, small_ids, first, count, cd, lds); break;
      case 6: seg_small_item<6>(keys, offsets, small_ids, first, count, cd, lds); break;
      default: seg_small_item<5>(keys, offsets, small_ids, first, count, cd, lds); break;
    }
  }
}

// ---------------------------------------------------------------------------
// big segments

// Largest i in [0, cnt) with prefix[i] <= v (prefix nondecreasing, prefix[0] = 0).
__device__ __forceinline__ uint32_t upper_index(const uint64_t* __restrict__ prefix, uint32_t cnt,
                                                uint64_t v) {
  uint32_t lo = 0, hi = cnt;  // answer in [lo, hi)
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (prefix[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

// A workgroup's share of `total` work units: the contiguous range
// [*first, *end), so that it searches the segment prefix sums once and then
// walks forward (a search per unit is ~11 dependent loads, which dominated
// the one-step passes).
__device__ __forceinline__ void unit_range(uint64_t total, uint64_t* first, uint64_t* end) {
  const uint64_t per = (total + gridDim.x - 1) / gridDim.x;
  const uint64_t a = (uint64_t)blockIdx.x * per;
  *first = a < total ? a : total;
  *end = a + per < total ? a + per : total;
}

// upper_index(prefix, cnt, v) given i = upper_index(prefix, cnt, v') for some
// v' <= v.
__device__ __forceinline__ uint32_t advance_index(const uint64_t* __restrict__ prefix,
                                                  uint32_t cnt, uint32_t i, uint64_t v) {
  while (i + 1 < cnt && prefix[i + 1] <= v) ++i;
  return i;
}

// Tile (log2 elements) and register slots (log2) per thread of the
// big-segment tile programs: 2^14 4-byte keys at 32 per thread; 2^13 8-byte
// elements at 16 per thread, so that a CU still runs 16 waves of them.
template <class ST>
constexpr int seg_tile_log() {
  return sizeof(typename ST::E) == 8 ? kSegTileLog64 : kSegTileLog32;
}
template <class ST>
constexpr int seg_tile_reg_log() {
  return sizeof(typename ST::E) == 8 ? 4 : kTileRegLogSeg;
}
template <class ST>
constexpr int seg_tile_threads() {
  return 1 << (seg_tile_log<ST>() - seg_tile_reg_log<ST>());
}

// Every tile of the big segments of class >= cls_min: sort (KIND 2 or 6) or
// merge (KIND 3).
template <int KIND, class ST, class CD>
__global__ __launch_bounds__(seg_tile_threads<ST>()) void seg_tile_kernel(
    ST keys, const int64_t* __restrict__ offsets,
    const SegMeta* __restrict__ meta, const uint32_t* __restrict__ big_ids,
    const uint64_t* __restrict__ big_tiles, int cls_min, CD cd) {
  using PR = Prog<seg_tile_log<ST>(), seg_tile_reg_log<ST>(), KIND>;
  static_assert(PR::NT == seg_tile_threads<ST>(), "one tile per workgroup");
  // 8-byte elements regroup through 4-byte words (half the LDS: four
  // workgroups per CU instead of two)
  constexpr bool SPLIT = sizeof(typename ST::E) == 8;
  __shared__ uint32_t lds32[PR::LDSW * (SPLIT ? 1 : sizeof(typename ST::E) / 4)];
  typename ST::E* lds = reinterpret_cast<typename ST::E*>(lds32);
  const uint32_t cnt = meta->big_ge[cls_min];
  uint64_t u, uend;
  unit_range(big_tiles[cnt], &u, &uend);
  uint32_t i = u < uend ? upper_index(big_tiles, cnt, u) : 0u;
  // tile uu's first element (segment-relative start off + t0) and its real
  // element count; i walks forward through the big-segment list
  auto locate = [&](uint64_t uu, uint64_t* start, uint32_t* valid) {
    i = advance_index(big_tiles, cnt, i, uu);
    const uint64_t tile = uu - big_tiles[i];
    const uint32_t s = big_ids[i];
    const int64_t off = offsets[s];
    const uint64_t len = (uint64_t)(offsets[s + 1] - off);
    const uint64_t t0 = tile << seg_tile_log<ST>();
    const uint64_t left = len - t0;
    *start = (uint64_t)off + t0;
    *valid = left < (uint64_t)PR::T ? (uint32_t)left : (uint32_t)PR::T;
  };
  if constexpr (std::is_same_v<ST, Keys32>) {
    // 4-byte keys: the next tile's keys are loaded (through a buffer
    // resource of its real keys, so slots past them read 0 and touch no
    // memory) while this tile is sorted and stored; each tile's keys are
    // encoded, and its padding set, only when its program starts.  The
    // sort runs a segment's last tile, when at most half of it holds keys,
    // with the half-size program (16 keys per thread, the same threads):
    // about 43 % of the work; that tile's keys are not prefetched.
    constexpr Group g0 = PR::value.g[0];
    constexpr int LAST = PR::value.ngroups - 1;
    constexpr bool HALF = KIND == 6;
    using PH = Prog<seg_tile_log<ST>() - 1, seg_tile_reg_log<ST>() - 1, KIND>;
    static_assert(!HALF || (PH::NT == PR::NT && PH::LDSW <= PR::LDSW), "half tile in the same workgroup");
    auto half = [](uint32_t v) { return HALF && v <= (uint32_t)PH::T; };
    auto load_raw = [&](int32_t (&x)[PR::R], uint64_t start, uint32_t valid, uint32_t tid) {
      const __amdgpu_buffer_rsrc_t rs = tile_rsrc(keys.k + start, valid * 4u);
      const uint32_t base = deposit<free_mask(g0, PR::L)>(tid);
      static_for<0, PR::R>([&](auto J) {
        const uint32_t idx = slot_index<PR, 0, J>(base);
        x[J] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, idx * 4u, 0, 0);
      });
    };
    if (u >= uend) return;
    uint64_t start = 0;
    uint32_t valid = 0;
    locate(u, &start, &valid);
    int32_t x[PR::R];
    load_raw(x, start, half(valid) ? 0u : valid, threadIdx.x);
    for (; u < uend; ++u) {
      uint32_t tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      uint64_t nstart = start;
      uint32_t nvalid = 0;  // no next tile: an empty resource
      if (u + 1 < uend) locate(u + 1, &nstart, &nvalid);
      int32_t y[PR::R];
      load_raw(y, nstart, half(nvalid) ? 0u : nvalid, tid);
      if (half(valid)) {
        tile_program<PH>(keys.k + start, valid, cd, lds, tid);  // loads its own keys
      } else {
        {
          const uint32_t base = deposit<free_mask(g0, PR::L)>(tid);
          static_for<0, PR::R>([&](auto J) {
            const uint32_t idx = slot_index<PR, 0, J>(base);
            x[J] = idx < valid ? cd.enc(x[J]) : kPad;
          });
        }
        run_from<PR, 0>(x, lds, tid);  // its first regroup waits for the LDS
        store_tile<PR, LAST>(x, keys.k + start, valid, cd, tid);
      }
      static_for<0, PR::R>([&](auto J) { x[J] = y[J]; });
      start = nstart;
      valid = nvalid;
    }
  } else {
    for (; u < uend; ++u) {
      // recompute the layouts' thread bases per tile instead of holding them
      uint32_t tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      uint64_t start = 0;
      uint32_t valid = 0;
      locate(u, &start, &valid);
      seg_tile_program<PR, SPLIT>(keys.at(start), valid, cd, lds, tid);
      __syncthreads();  // LDS reuse by the next tile
    }
  }
}

// Phase T + 1 of the big segments of that class and above (T the big
// segments' tile, seg_tile_log): the mirror step and the half-cleaners on
// units of 2^(T+1) elements, whose two halves the tile sort left ascending
// (program kind 7, scalar I/O).  Units run over the segments' padded sizes
// (big_keys), so a unit wholly in a segment's virtual padding has no work
// and is skipped; each workgroup takes a contiguous range of units (one per
// CU for 4-byte keys, 135 KiB of LDS; two for 8-byte elements, whose
// regroups go through 4-byte words).  For 4-byte keys the next unit's keys
// are loaded (through a buffer resource of its real keys) while this one is
// processed.
template <class ST>
constexpr int seg_phase_log() {
  return seg_tile_log<ST>() + 1;
}
template <class ST>
constexpr int seg_phase_threads() {
  return 1 << (seg_phase_log<ST>() - seg_tile_reg_log<ST>());
}

template <class ST, class CD>
__global__ __launch_bounds__(seg_phase_threads<ST>()) void seg_phase_kernel(
    ST keys, const int64_t* __restrict__ offsets, const SegMeta* __restrict__ meta,
    const uint32_t* __restrict__ big_ids, const uint64_t* __restrict__ big_keys, CD cd) {
  constexpr int kSegPhaseLog = seg_phase_log<ST>();
  using PR = Prog<kSegPhaseLog, seg_tile_reg_log<ST>(), 7>;
  static_assert(PR::NT == seg_phase_threads<ST>(), "one unit per workgroup");
  constexpr bool SPLIT = sizeof(typename ST::E) == 8;
  __shared__ uint32_t lds32[PR::LDSW];
  constexpr Group g0 = PR::value.g[0];
  constexpr int LAST = PR::value.ngroups - 1;
  const uint32_t cnt = meta->big_ge[kSegPhaseLog];
  uint64_t u, uend;
  unit_range(big_keys[cnt] >> kSegPhaseLog, &u, &uend);
  uint32_t i = u < uend ? upper_index(big_keys, cnt, u << kSegPhaseLog) : 0u;
  // unit uu's first element and real element count; false for a unit of
  // padding only (the same answer for the whole workgroup)
  auto locate = [&](uint64_t uu, uint64_t* start, uint32_t* valid) -> bool {
    const uint64_t key0 = uu << kSegPhaseLog;
    i = advance_index(big_keys, cnt, i, key0);
    const uint64_t lk = key0 - big_keys[i];  // unit's first element, segment-local
    const uint32_t s = big_ids[i];
    const int64_t off = offsets[s];
    const uint64_t len = (uint64_t)(offsets[s + 1] - off);
    if (lk >= len) return false;
    const uint64_t left = len - lk;
    *start = (uint64_t)off + lk;
    *valid = left < (uint64_t)PR::T ? (uint32_t)left : (uint32_t)PR::T;
    return true;
  };
  uint64_t start = 0;
  uint32_t valid = 0;
  if constexpr (SPLIT) {
    for (; u < uend; ++u) {
      if (!locate(u, &start, &valid)) continue;
      uint32_t tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      seg_tile_program<PR, true>(keys.at(start), valid, cd,
                                 reinterpret_cast<typename ST::E*>(lds32), tid);
      __syncthreads();  // LDS reuse by the next unit
    }
  } else {
    int32_t* lds = reinterpret_cast<int32_t*>(lds32);
    auto load_raw = [&](int32_t (&x)[PR::R], uint64_t st0, uint32_t v, uint32_t tid) {
      const __amdgpu_buffer_rsrc_t rs = tile_rsrc(keys.k + st0, v * 4u);
      const uint32_t base = deposit<free_mask(g0, PR::L)>(tid);
      static_for<0, PR::R>([&](auto J) {
        const uint32_t idx = slot_index<PR, 0, J>(base);
        x[J] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rs, idx * 4u, 0, 0);
      });
    };
    while (u < uend && !locate(u, &start, &valid)) ++u;
    if (u >= uend) return;
    int32_t x[PR::R];
    load_raw(x, start, valid, threadIdx.x);
    while (u < uend) {
      uint32_t tid = threadIdx.x;
      asm volatile("" : "+v"(tid));
      uint64_t nu = u + 1;
      uint64_t nstart = start;
      uint32_t nvalid = 0;  // no next unit: an empty resource
      while (nu < uend && !locate(nu, &nstart, &nvalid)) ++nu;
      int32_t y[PR::R];
      load_raw(y, nstart, nvalid, tid);
      {
        const uint32_t base = deposit<free_mask(g0, PR::L)>(tid);
        static_for<0, PR::R>([&](auto J) {
          const uint32_t idx = slot_index<PR, 0, J>(base);
          x[J] = idx < valid ? cd.enc(x[J]) : kPad;
        });
      }
      run_from<PR, 0>(x, lds, tid);  // its first regroup waits for the LDS
      store_tile<PR, LAST>(x, keys.k + start, valid, cd, tid);
      static_for<0, PR::R>([&](auto J) { x[J] = y[J]; });
      start = nstart;
      valid = nvalid;
      u = nu;
    }
  }
}

// Columns per thread of a big-segment pass of F steps: 4 up to F = 3, then
// fewer as the rows double, so that a thread holds at most 32 elements
// (2^F rows x the columns).
constexpr int seg_pass_cols(int F) { return F <= 3 ? 4 : (F == 4 ? 2 : 1); }
constexpr int seg_pass_cols_log(int F) { return F <= 3 ? 2 : (F == 4 ? 1 : 0); }

// Segment-local index of register slot (RHO, J) of a pass unit: row RHO of
// the block at blk, column c0 + threadIdx.x + 256 J (mirrored rows: the
// mirror image inside the block).
template <int F, bool MIRROR, int RHO, int J>
__device__ __forceinline__ uint32_t seg_pass_index(uint32_t blk, uint32_t c0, int q) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  const uint32_t col = c0 + threadIdx.x + 256u * (uint32_t)J;
  if constexpr (MIRROR && (RHO & TOP))
    return blk + ((uint32_t)((ROWS - 1) ^ (RHO & (TOP - 1))) << q) + (((1u << q) - 1u) - col);
  else
    return blk + ((uint32_t)RHO << q) + col;
}

// F fused long-stride steps (bits q+F-1 .. q, F <= kSegFuseMax) over the big
// segments of class >= cls.  A workgroup unit is 256 C consecutive columns x
// 2^F rows of one 2^(q+F)-element block of one segment (C = seg_pass_cols(F));
// thread t holds columns c0 + t + 256 j (j < C), so every load and store of
// a wave is 64 consecutive elements.  Since q is at least the tile's log2
// (13 or 14), a block holds whole units.
template <int F, bool MIRROR, class ST, class CD>
__global__ __launch_bounds__(kSegThreads) void seg_pass_kernel(
    ST keys, const int64_t* __restrict__ offsets,
    const SegMeta* __restrict__ meta, const uint32_t* __restrict__ big_ids,
    const uint64_t* __restrict__ big_keys, int cls, int q, CD cd) {
  constexpr int ROWS = 1 << F;
  constexpr int COLS = seg_pass_cols(F);
  constexpr int COL_LOG = 8 + seg_pass_cols_log(F);  // columns per unit, log2
  constexpr int UNIT_LOG = COL_LOG + F;              // elements per unit, log2
  const uint32_t cnt = meta->big_ge[cls];
  uint64_t u, uend;
  unit_range(big_keys[cnt] >> UNIT_LOG, &u, &uend);
  uint32_t i = u < uend ? upper_index(big_keys, cnt, u << UNIT_LOG) : 0u;
  for (; u < uend; ++u) {
    const uint64_t key0 = u << UNIT_LOG;
    i = advance_index(big_keys, cnt, i, key0);
    const uint64_t lk = key0 - big_keys[i];  // unit's first key, segment-local
    const uint32_t s = big_ids[i];
    const int64_t off = offsets[s];
    const uint32_t len = (uint32_t)(offsets[s + 1] - off);
    const ST a = keys.at(off);
    // unit -> block and column run: a block holds 2^(q - COL_LOG) units;
    // segment-local indices fit 32 bits (segments hold < 2^31 keys)
    const uint32_t lu = (uint32_t)(lk >> UNIT_LOG);
    const int upb_log = q - COL_LOG;
    const uint32_t blk = (lu >> upb_log) << (q + F);
    const uint32_t c0 = (lu & ((1u << upb_log) - 1u)) << COL_LOG;
    typename ST::E x[COLS * ROWS];
    static_for<0, ROWS>([&](auto RHO) {
      static_for<0, COLS>([&](auto J) {
        const uint32_t idx = seg_pass_index<F, MIRROR, RHO, J>(blk, c0, q);
        x[COLS * RHO + J] = idx < len ? cd.enc(a.get(idx)) : ST::kPadE;
      });
    });
    pass_steps<F, MIRROR, COLS>(x);
    static_for<0, ROWS>([&](auto RHO) {
      static_for<0, COLS>([&](auto J) {
        const uint32_t idx = seg_pass_index<F, MIRROR, RHO, J>(blk, c0, q);
        if (idx < len) a.put(idx, cd.dec(x[COLS * RHO + J]));
      });
    });
  }
}

// ---------------------------------------------------------------------------
// launch of one kernel of the sequence (SegLaunch) on a storage

template <class ST, class CD>
void seg_run(ST keys, CD cd, const SegLaunch& l, const int64_t* offsets, const SegScratch& sc,
             hipStream_t st) {
  switch (l.what) {
    case SegLaunch::kSmall:
      seg_small_kernel<<<l.grid, kSegThreads, 0, st>>>(keys, offsets, sc.meta, sc.small_ids, cd);
      break;
    case SegLaunch::kTileSort:
      seg_tile_kernel<seg_sort_kind<ST>()><<<l.grid, seg_tile_threads<ST>(), 0, st>>>(
          keys, offsets, sc.meta, sc.big_ids, sc.big_tiles, l.cls, cd);
      break;
    case SegLaunch::kTileMerge:
      seg_tile_kernel<3><<<l.grid, seg_tile_threads<ST>(), 0, st>>>(
          keys, offsets, sc.meta, sc.big_ids, sc.big_tiles, l.cls, cd);
      break;
    case SegLaunch::kPhase:
      seg_phase_kernel<<<l.grid, seg_phase_threads<ST>(), 0, st>>>(keys, offsets, sc.meta,
                                                                   sc.big_ids, sc.big_keys, cd);
      break;
    case SegLaunch::kPass: {
#define BITONIC_SEG_PASS(F)                                                                     \
  if (l.mirror)                                                                                 \
    seg_pass_kernel<F, true><<<l.grid, kSegThreads, 0, st>>>(keys, offsets, sc.meta, sc.big_ids, \
                                                             sc.big_keys, l.cls, l.q, cd);      \
  else                                                                                          \
    seg_pass_kernel<F, false><<<l.grid, kSegThreads, 0, st>>>(keys, offsets, sc.meta,           \
                                                              sc.big_ids, sc.big_keys, l.cls,   \
                                                              l.q, cd);
      if (l.f == 1) { BITONIC_SEG_PASS(1) }
      else if (l.f == 2) { BITONIC_SEG_PASS(2) }
      else if (l.f == 3) { BITONIC_SEG_PASS(3) }
      else if (l.f == 4) { BITONIC_SEG_PASS(4) }
      else if (l.f == 5) { BITONIC_SEG_PASS(5) }
      static_assert(kSegFuseMax == 5, "one instantiation per fused step count");
#undef BITONIC_SEG_PASS
      break;
    }
    default:
      break;
  }
}

}  // namespace bitonic
