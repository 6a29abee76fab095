// Segmented sort: many independent arrays described by a CSR offset table.
// Every segment of length len runs the flip network of the single-array sort
// on its own padded size 2^m (m = ceil(log2 len), its "class"), with the keys
// past len left virtual.
//
// Launch sequence (all on one stream, no host synchronisation):
//   seg_prep_kernel      one workgroup classifies the segments: class
//                        counts, segment ids bucketed by class (largest
//                        first), prefix sums over the big segments
//   seg_small_kernel     persistent; every work item is up to 256 / 2^(m-5)
//                        segments of one class m <= 13, each sorted by its own
//                        group of threads with the register tile programs
//                        (scalar I/O, group-private LDS region); items are
//                        taken from an atomic counter, largest class first
//   seg_tile_kernel      tile sort of every tile of the big segments (class
//                        > 13; 2^14-key tiles for 4-byte keys, 2^13-element
//                        for 8-byte elements), over a device-side tile list
//   seg_pass_kernel and  per phase p above the tile: the fused long-stride
//   seg_tile_kernel      steps and the tile merges of the big segments of
//                        class >= p
// The host only needs an upper bound on the largest class to know how many
// phases to enqueue.
#include "seg_kernels.hpp"

namespace bitonic {

// ---------------------------------------------------------------------------
// validation (only when enabled: bitonic_set_tuning_value("validate", 1) or
// BITONIC_VALIDATE=1)

// First table error any validated call found on this device (0: none).
__device__ int32_t g_seg_validation_error;

__global__ __launch_bounds__(1024) void seg_validate_kernel(const int64_t* __restrict__ offsets,
                                                            int64_t nseg, int64_t bound,
                                                            SegMeta* __restrict__ meta) {
  __shared__ int32_t err;
  if (threadIdx.x == 0) err = offsets[0] < 0 ? kSegTableNegative : kSegTableOk;
  __syncthreads();
  for (int64_t s = threadIdx.x; s < nseg; s += 1024) {
    const int64_t len = offsets[s + 1] - offsets[s];
    int32_t e = kSegTableOk;
    if (len < 0) e = kSegTableDecreasing;
    else if (len >= (int64_t(1) << 31)) e = kSegTableTooLong;
    else if (len > bound) e = kSegTableOverBound;
    if (e != kSegTableOk) atomicCAS(&err, kSegTableOk, e);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    meta->invalid = err;
    if (err != kSegTableOk) atomicCAS(&g_seg_validation_error, kSegTableOk, err);
  }
}

void launch_seg_validate(const int64_t* offsets, int64_t nseg, int64_t bound, const SegScratch& sc,
                         hipStream_t st) {
  seg_validate_kernel<<<1, 1024, 0, st>>>(offsets, nseg, bound, sc.meta);
}

int seg_validation_error(int32_t* code) {
  int32_t v = 0;
  const int32_t zero = 0;
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpyFromSymbol(&v, HIP_SYMBOL(g_seg_validation_error), sizeof v) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(g_seg_validation_error), &zero, sizeof zero) != hipSuccess)
    return -1;
  *code = v;
  return 0;
}

// ---------------------------------------------------------------------------
// prep

__global__ __launch_bounds__(1024) void seg_prep_kernel(const int64_t* __restrict__ offsets,
                                                        int64_t nseg, SegMeta* __restrict__ meta,
                                                        uint32_t* __restrict__ small_ids,
                                                        uint32_t* __restrict__ big_ids,
                                                        uint64_t* __restrict__ big_keys,
                                                        uint64_t* __restrict__ big_tiles,
                                                        int tile_log, int validated) {
  __shared__ uint32_t cnt[32];
  __shared__ uint32_t cur[32];
  __shared__ uint64_t part_k[1024];
  __shared__ uint64_t part_t[1024];
  __shared__ uint32_t nbig_s;
  const uint32_t tid = threadIdx.x;
  if (validated && meta->invalid) {
    // a refused table classifies as empty: no kernel after this one touches
    // the keys or reads the offsets again
    if (tid == 0) {
      meta->small_counter = 0;
      meta->small_items = 0;
      meta->nbig = 0;
      meta->max_class = 0;
      for (int i = 0; i < kSmallClasses; ++i) {
        meta->small_start[i] = 0;
        meta->small_count[i] = 0;
        meta->item_prefix[i] = 0;
      }
      meta->item_prefix[kSmallClasses] = 0;
      for (int c = 0; c < 33; ++c) meta->big_ge[c] = 0;
      big_keys[0] = 0;
      big_tiles[0] = 0;
    }
    return;
  }
  if (tid < 32) cnt[tid] = 0;
  __syncthreads();
  for (int64_t s = tid; s < nseg; s += 1024) {
    const uint64_t len = (uint64_t)(offsets[s + 1] - offsets[s]);
    if (len <= 1) continue;
    int c = ceil_log2_u64(len);
    if (c < 5) c = 5;
    atomicAdd(&cnt[c], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    // small buckets, class 13 first
    uint32_t pos = 0, items = 0;
    for (int i = 0; i < kSmallClasses; ++i) {
      const int c = small_class_of_index(i);
      meta->small_start[i] = pos;
      meta->small_count[i] = cnt[c];
      meta->item_prefix[i] = items;
      cur[c] = pos;
      pos += cnt[c];
      const uint32_t per = small_per_item(c);
      items += (cnt[c] + per - 1) / per;
    }
    meta->item_prefix[kSmallClasses] = items;
    meta->small_items = items;
    meta->small_counter = 0;
    // big buckets, largest class first
    uint32_t bpos = 0;
    int maxc = 0;
    for (int c = 31; c > kSegSmallMaxLog2; --c) {
      cur[c] = bpos;
      bpos += cnt[c];
      meta->big_ge[c] = bpos;  // segments of class >= c
      if (cnt[c] && !maxc) maxc = c;
    }
    for (int c = 0; c <= kSegSmallMaxLog2; ++c) meta->big_ge[c] = bpos;
    meta->big_ge[32] = 0;
    meta->nbig = bpos;
    meta->max_class = maxc;
    nbig_s = bpos;
  }
  __syncthreads();
  for (int64_t s = tid; s < nseg; s += 1024) {
    const uint64_t len = (uint64_t)(offsets[s + 1] - offsets[s]);
    if (len <= 1) continue;
    int c = ceil_log2_u64(len);
    if (c < 5) c = 5;
    const uint32_t slot = atomicAdd(&cur[c], 1u);
    if (c <= kSegSmallMaxLog2)
      small_ids[slot] = (uint32_t)s;
    else
      big_ids[slot] = (uint32_t)s;
  }
  __syncthreads();
  // exclusive prefix sums over the big list (padded keys, real tiles)
  const uint32_t nbig = nbig_s;
  const uint32_t chunk = (nbig + 1023) / 1024;
  const uint32_t b0 = tid * chunk;
  const uint32_t b1 = min(b0 + chunk, nbig);
  uint64_t sk = 0, st = 0;
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t s = big_ids[i];
    const uint64_t len = (uint64_t)(offsets[s + 1] - offsets[s]);
    sk += 1ull << ceil_log2_u64(len);
    st += (len + (1ull << tile_log) - 1) >> tile_log;
  }
  part_k[tid] = sk;
  part_t[tid] = st;
  __syncthreads();
  // inclusive scan of the 1024 chunk sums (ten rounds of adding the sum d
  // places back, d = 1, 2, 4, ...), then each chunk's exclusive start
  for (uint32_t d = 1; d < 1024; d <<= 1) {
    const uint64_t ak = tid >= d ? part_k[tid - d] : 0;
    const uint64_t at = tid >= d ? part_t[tid - d] : 0;
    __syncthreads();
    part_k[tid] += ak;
    part_t[tid] += at;
    __syncthreads();
  }
  if (tid == 1023) {
    big_keys[nbig] = part_k[tid];
    big_tiles[nbig] = part_t[tid];
  }
  sk = part_k[tid] - sk;
  st = part_t[tid] - st;
  for (uint32_t i = b0; i < b1; ++i) {
    const uint32_t s = big_ids[i];
    const uint64_t len = (uint64_t)(offsets[s + 1] - offsets[s]);
    big_keys[i] = sk;
    big_tiles[i] = st;
    sk += 1ull << ceil_log2_u64(len);
    st += (len + (1ull << tile_log) - 1) >> tile_log;
  }
}

// ---------------------------------------------------------------------------
// launchers: dispatch on the data of the sort to its storage's instantiation

static void seg_dispatch(const SegData& d, const SegLaunch& l, const int64_t* offsets,
                         const SegScratch& sc, hipStream_t st) {
  if (d.keys64)
    seg_run_keys64(d, l, offsets, sc, st);
  else if (d.values)
    seg_run_pairs(d, l, offsets, sc, st);
  else
    seg_run_keys32(d, l, offsets, sc, st);
}

void launch_seg_prep(const int64_t* offsets, int64_t nseg, const SegScratch& sc, int tile_log,
                     bool validated, hipStream_t st) {
  seg_prep_kernel<<<1, 1024, 0, st>>>(offsets, nseg, sc.meta, sc.small_ids, sc.big_ids,
                                      sc.big_keys, sc.big_tiles, tile_log, validated ? 1 : 0);
}

void launch_seg_small(const SegData& d, const int64_t* offsets, const SegScratch& sc, int grid,
                      hipStream_t st) {
  SegLaunch l{};
  l.what = SegLaunch::kSmall;
  l.grid = grid;
  seg_dispatch(d, l, offsets, sc, st);
}

void launch_seg_tiles(bool merge, const SegData& d, const int64_t* offsets, const SegScratch& sc,
                      int cls_min, int grid, hipStream_t st) {
  SegLaunch l{};
  l.what = merge ? SegLaunch::kTileMerge : SegLaunch::kTileSort;
  l.cls = cls_min;
  l.grid = grid;
  seg_dispatch(d, l, offsets, sc, st);
}

void launch_seg_phase(const SegData& d, const int64_t* offsets, const SegScratch& sc, int grid,
                      hipStream_t st) {
  SegLaunch l{};
  l.what = SegLaunch::kPhase;
  l.grid = grid;
  seg_dispatch(d, l, offsets, sc, st);
}

void launch_seg_pass(int f, bool mirror, const SegData& d, const int64_t* offsets,
                     const SegScratch& sc, int cls, int q, int grid, hipStream_t st) {
  SegLaunch l{};
  l.what = SegLaunch::kPass;
  l.f = f;
  l.mirror = mirror;
  l.cls = cls;
  l.q = q;
  l.grid = grid;
  seg_dispatch(d, l, offsets, sc, st);
}

}  // namespace bitonic
