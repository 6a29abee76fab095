// Planners and C interface (include/bitonic.h): single-array sorts of 4-byte
// keys, of 8-byte keys and of (key, value) pairs, the segmented sort, graph
// capture, tuning.
//
// The planner maps the k(k+1)/2 steps of the network for N = 2^k keys
// (sections 3.2, 3.3) onto kernel launches, all enqueued on the caller's
// stream with no host synchronisation:
//   optimized: one tile sort (phases 1..t), then for each phase p > t the
//              p - t long-stride steps in ceil((p - t) / f) fused HBM passes
//              followed by one tile merge (strides 2^(t-1)..1);
//   semi:      LDS tile network for phases 1..t, one launch per long-stride
//              step, one LDS tail per phase (section 4.1 alone);
//   basic:     one launch per step (section 3.3).
// The 8-byte sorts use the optimized plan on 8-byte elements (enqueue_wide);
// the segmented sort classifies its segments on the device and runs the
// optimized plan's structure per class (enqueue_segmented).
#include <atomic>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "bitonic.h"
#include "launch.hpp"
#include "scratch_cache.hpp"
#include "segmented.hpp"

namespace bitonic {

static std::atomic<int> g_tile_log2{0};  // 0: by n (default_tile_log2)
static std::atomic<int> g_fuse{10};
static std::atomic<int> g_merge_bpc{2};  // 0: one tile per workgroup
static std::atomic<int> g_wide_tile_log2{13};  // 8-byte sorts
static std::atomic<int> g_wide_fuse{8};
static std::atomic<int> g_seg_bpc{4};    // small-segment workgroups per compute unit
static std::atomic<int> g_seg_pass_bpc{8};  // big-segment pass workgroups per compute unit
static std::atomic<int> g_seg_fuse{kSegFuseMax};  // steps per big-segment pass
static std::atomic<int> g_tile_lane{1};  // tile sort with cross-lane steps (program kind 4)
// Lane passes (columns split over lanes; launch_column_lanes_pass): 0 off, so
// at most kFuseMaxColumn steps per pass; 8: nine and ten steps as 2^8 keys
// per lane over two and four lanes; 7: eight and nine steps as 2^7 keys per
// lane over two and four lanes (ten as with 8).
static std::atomic<int> g_lane_pass{7};
// Phase t+1 of a sort with 2^t-key tiles (t <= 14) as one tile-phase launch
// on 2^(t+1)-key tiles instead of a one-step pass and a merge.
static std::atomic<int> g_phase_merge{1};
// Tile-phase workgroups per compute unit, each looping over its tiles
// (-1: one tile per workgroup; 0: as the tile merges).
static std::atomic<int> g_phase_bpc{1};
// Tile-sort tile (log2 keys) of the optimized plan when larger than the
// merge tile, for n a power of two: phases 1..s sort in one launch, later
// phases pass down to the merge tile's bit and merge 2^t-key tiles (0: the
// merge tile).
static std::atomic<int> g_sort_tile{0};
static std::atomic<int> g_validate{-1};  // check segment tables on the device; -1: not yet read

// Offsets validation of the segmented sorts: the tuning value "validate", or
// else the environment variable BITONIC_VALIDATE=1.
static bool validate_enabled() {
  int v = g_validate.load();
  if (v < 0) {
    const char* e = std::getenv("BITONIC_VALIDATE");
    v = (e && e[0] == '1' && e[1] == 0) ? 1 : 0;
    int expect = -1;
    g_validate.compare_exchange_strong(expect, v);
    v = g_validate.load();
  }
  return v == 1;
}

struct Resolved {
  int kind;
  int tile;
  int sort_tile = 0;      // tile sort's tile (log2), >= tile (optimized plan)
  int fuse;
  int sort_kind = 0;      // tile-sort program: 0, or 4 with cross-lane steps
  int merge_bpc;          // tile-merge workgroups per compute unit
  int lane_pass = 0;      // g_lane_pass at resolve time
  bool phase_merge = false;  // g_phase_merge at resolve time
  uint32_t merge_blocks;  // merge_bpc x compute units (set when enqueueing)
  uint32_t phase_blocks = 0;  // the same for the tile phase
  bool scalar_io = false;  // optimized plan for an array off a 16-byte boundary
};

// The library's tile size for n keys (measured on MI355X: below 2^21 keys
// smaller tiles give more workgroups than the 256 CUs need, above it the
// larger tile's fewer launches win).
static int default_tile_log2(int64_t n) {
  int k = 0;
  while ((int64_t(1) << k) < n) ++k;
  return k <= 16 ? 12 : (k <= 20 ? 13 : 14);
}

static int ceil_log2(int64_t n) {
  int k = 0;
  while ((int64_t(1) << k) < n) ++k;
  return k;
}

// Tuned plans by size bucket k = ceil(log2 n) (tuning keys "tile_log2@k",
// "fuse@k", "merge_blocks_per_cu@k", "lane_pass@k"; 0 = no entry).  A bucket's entries take
// precedence over the global tuning values, an explicit plan over both.
constexpr int kBuckets = 32;
static std::atomic<int> g_bk_tile[kBuckets];
static std::atomic<int> g_bk_fuse[kBuckets];
static std::atomic<int> g_bk_merge[kBuckets];  // -1: one tile per workgroup
static std::atomic<int> g_bk_lane[kBuckets];   // lane-pass mode (7, 8, 9)
static std::atomic<int> g_bk_sort_tile[kBuckets];  // tile-sort tile (log2)

// The tuning file named by the environment variable BITONIC_TUNE_FILE, if
// any, is loaded once, before the first plan is resolved.
static void load_env_tuning_once() {
  static std::once_flag once;
  std::call_once(once, [] {
    const char* p = std::getenv("BITONIC_TUNE_FILE");
    if (p && *p) (void)bitonic_load_tuning(p);
  });
}

static int resolve(const bitonic_plan* plan, int64_t n, Resolved* r) {
  load_env_tuning_once();
  r->kind = BITONIC_PLAN_OPTIMIZED;
  r->tile = g_tile_log2.load();
  r->fuse = g_fuse.load();
  r->merge_bpc = g_merge_bpc.load();
  r->merge_blocks = 0;
  r->sort_kind = g_tile_lane.load() ? 4 : 0;
  r->lane_pass = g_lane_pass.load();
  int sort_tile = g_sort_tile.load();
  {
    const int k = n > (int64_t(1) << 31) ? 31 : ceil_log2(n < 1 ? 1 : n);
    if (const int t = g_bk_tile[k].load()) r->tile = t;
    if (const int f = g_bk_fuse[k].load()) r->fuse = f;
    if (const int m = g_bk_merge[k].load()) r->merge_bpc = m > 0 ? m : 0;
    if (const int lp = g_bk_lane[k].load()) r->lane_pass = lp;
    if (const int s = g_bk_sort_tile[k].load()) sort_tile = s;
  }
  if (plan) {
    if (plan->kind < BITONIC_PLAN_AUTO || plan->kind > BITONIC_PLAN_OPTIMIZED) return BITONIC_EINVAL;
    if (plan->merge_blocks_per_cu < -1 || plan->merge_blocks_per_cu > 16) return BITONIC_EINVAL;
    if (plan->kind != BITONIC_PLAN_AUTO) r->kind = plan->kind;
    if (plan->tile_log2) r->tile = plan->tile_log2;
    if (plan->fuse) r->fuse = plan->fuse;
    if (plan->merge_blocks_per_cu > 0) r->merge_bpc = plan->merge_blocks_per_cu;
    if (plan->merge_blocks_per_cu < 0) r->merge_bpc = 0;
  }
  if (r->kind == BITONIC_PLAN_SEMI) {
    if (!plan || !plan->tile_log2) r->tile = 12;
    if (r->tile < 1 || r->tile > kLdsNetworkMaxLog2) return BITONIC_EINVAL;
  }
  if (r->kind == BITONIC_PLAN_OPTIMIZED && r->tile == 0) r->tile = default_tile_log2(n);
  if (r->kind == BITONIC_PLAN_OPTIMIZED && !tile_log2_supported(r->tile)) return BITONIC_EINVAL;
  // Larger tile sorts only for powers of two (measured on MI355X: 2^15-key
  // tile sorts ahead of 2^14-key merges make n = 2^24 1 % faster, n = 10^7
  // 2 % slower).
  r->sort_tile = r->kind == BITONIC_PLAN_OPTIMIZED && sort_tile > r->tile && (n & (n - 1)) == 0
                     ? sort_tile : r->tile;
  if (r->fuse < 1 || r->fuse > kFuseMax) return BITONIC_EINVAL;
  r->phase_merge = g_phase_merge.load() != 0;
  return BITONIC_OK;
}

// Receives every launch of a plan as it is enqueued (or counted).
struct Observer {
  int32_t* kinds = nullptr;   // launch kind per launch (bitonic_launch_kind)
  int32_t* fuse = nullptr;    // fused steps per launch (global passes), else 0
  bitonic_launch_shape* shapes = nullptr;  // full shape per launch
  int64_t cap = 0;
  hipEvent_t* events = nullptr;  // events[i + 1] recorded after launch i
  int64_t nevents = 0;
  int64_t first = 0;             // only launches [first, first + count) run
  int64_t count = INT64_MAX;
};

// Keys per lane (log2) of an f-step lane pass under lane-pass mode `mode`
// (g_lane_pass), or 0 for a register pass; negative: the column spread over
// the four waves of a workgroup (column_waves_pass_kernel) with 2^-fr keys
// per lane.
static int lane_pass_regs(int mode, int f) {
  if (mode == 8) return f >= 9 ? 8 : 0;
  if (mode == 7) return f == 8 || f == 9 ? 7 : (f == 10 ? 8 : 0);
  if (mode == 9) return f == 8 ? 7 : (f == 9 ? -7 : (f == 10 ? -8 : 0));
  return 0;
}

// Enqueue (or, with count_only, just count) the launches for phases 1..K of
// the network over keys[0, n).
static int64_t enqueue_plain(int32_t* keys, uint32_t n, int K, Codec flip, const Resolved& r,
                             hipStream_t st, bool count_only, Observer* obs = nullptr) {
  const int k = ceil_log2(n);
  const uint32_t N = (k >= 32) ? 0u : (1u << k);
  int64_t launches = 0;
  if (K > k) K = k;
  if (K <= 0) return 0;
  // every launch is described by its shape (bitonic_plan_shapes); the
  // 4-byte kernels index elements through 64-bit pointers except the fused
  // passes, whose lane byte offsets are 32-bit (column_pass_offset_bits)
  auto emit = [&](bitonic_launch_shape sh, auto&& launch) {
    const bool selected =
        !obs || (launches >= obs->first && launches - obs->first < obs->count);
    if (!count_only && selected) launch();
    if (obs) {
      if (launches < obs->cap) {
        if (obs->kinds) obs->kinds[launches] = sh.kind;
        if (obs->fuse) obs->fuse[launches] = sh.fuse;
        if (obs->shapes) obs->shapes[launches] = sh;
      }
      if (!count_only && obs->events && launches + 1 < obs->nevents)
        (void)hipEventRecord(obs->events[launches + 1], st);
    }
    ++launches;
  };
  if (obs && !count_only && obs->events && obs->nevents > 0)
    (void)hipEventRecord(obs->events[0], st);

  auto step_shape = [](int sb, bool mirror) {
    return bitonic_launch_shape{BITONIC_LAUNCH_STEP, 1, sb, mirror ? 1 : 0, 4, 64};
  };
  auto tile_shape = [](int kind, int L) { return bitonic_launch_shape{kind, 0, L, 0, 4, 64}; };

  if (r.kind == BITONIC_PLAN_BASIC) {
    for (int p = 1; p <= K; ++p)
      for (int sb = p - 1; sb >= 0; --sb)
        emit(step_shape(sb, sb == p - 1),
             [&] { launch_step(sb, sb == p - 1, keys, n, N, flip, st); });
    return launches;
  }

  if (r.kind == BITONIC_PLAN_SEMI) {
    const int L = K < r.tile ? K : r.tile;
    emit(tile_shape(BITONIC_LAUNCH_LDS_NETWORK, L),
         [&] { launch_lds_network(L, 1, L, false, keys, n, flip, st); });
    for (int p = L + 1; p <= K; ++p) {
      for (int sb = p - 1; sb >= L; --sb)
        emit(step_shape(sb, sb == p - 1),
             [&] { launch_step(sb, sb == p - 1, keys, n, N, flip, st); });
      emit(tile_shape(BITONIC_LAUNCH_LDS_NETWORK, L),
           [&] { launch_lds_network(L, 0, 0, true, keys, n, flip, st); });
    }
    return launches;
  }

  // optimized
  if (K <= r.sort_tile) {
    // Phases 1..K.  The scalar-access tile sorts 2^13-key tiles, which is
    // phases 1..K only when one tile holds all n keys (K == k); fewer phases
    // of a longer array run in the LDS network.
    if (K < kTileMinLog2 || (r.scalar_io && K < kScalarTileLog2 && K < k))
      emit(tile_shape(BITONIC_LAUNCH_LDS_NETWORK, K),
           [&] { launch_lds_network(K, 1, K, false, keys, n, flip, st); });
    else if (r.scalar_io)
      emit(tile_shape(BITONIC_LAUNCH_TILE_SORT, kScalarTileLog2),
           [&] { launch_tile_scalar(0, keys, n, flip, CX_BOTH, st); });
    else
      emit(tile_shape(BITONIC_LAUNCH_TILE_SORT, K),
           [&] { launch_tile(K, r.sort_kind, keys, n, flip, CX_BOTH, 0, st); });
    return launches;
  }
  // The tile sort encodes the keys and the last merge decodes them; the
  // passes and merges in between work on encoded keys.  The tile sort takes
  // phases 1..Ls; each later phase passes down to bit L and merges 2^L-key
  // tiles (Ls >= L).
  const int L = r.tile;
  const int Ls = r.sort_tile;
  // Passes of more than kFuseMaxColumn steps split each column over lanes
  // (or waves); they need lane byte offsets below 2^32 (lane_pass_fits):
  // arrays on a 16-byte boundary, phases up to 30.  When n is not a power of
  // two the block of a pass that straddles n is bounds-checked: the lane
  // passes (lane mode 7's mapping, since the wave passes need whole blocks)
  // take eight to ten steps, while the one-column pass would take eight
  // only with more registers than it has, so without lane passes such sorts
  // use at most seven.
  const bool ragged = (n & (n - 1)) != 0;
  const bool lanes_ok = r.lane_pass != 0 && !r.scalar_io;
  const int lane_mode = ragged ? 7 : r.lane_pass;
  emit(tile_shape(BITONIC_LAUNCH_TILE_SORT, Ls), [&] {
    if (r.scalar_io)
      launch_tile_scalar(0, keys, n, flip, CX_ENC, st);
    else
      launch_tile(Ls, r.sort_kind, keys, n, flip, CX_ENC, 0, st);
  });
  for (int p = Ls + 1; p <= K; ++p) {
    if (p == Ls + 1 && r.phase_merge && !r.scalar_io && p <= kTileMaxLog2) {
      // the whole phase on 2^p-key tiles (mirror step included)
      const int cx = p == K ? CX_DEC : CX_NONE;
      emit(bitonic_launch_shape{BITONIC_LAUNCH_TILE_MERGE, 0, p, 1, 4, 64},
           [&] { launch_tile(p, 5, keys, n, flip, cx, r.phase_blocks, st); });
      continue;
    }
    const bool lanes = lanes_ok && p <= 30;
    const int cap = lanes ? kFuseMax : (ragged ? kFuseMaxRagged : kFuseMaxColumn);
    const int fz = r.fuse < cap ? r.fuse : cap;
    const int nb = p - L;                          // long-stride steps
    const int npass = (nb + fz - 1) / fz;          // fused HBM passes
    int top = p - 1;
    // Each pass takes as many steps as it may, the last one what is left:
    // the phase's first pass, the one with the mirror step, is then always
    // the widest (measured: a mirror pass of few steps over strides of
    // 2^17 or more runs up to 50 % slower than one of five).
    for (int i = 0; i < npass; ++i) {
      const int left = top - L + 1;                // bits still to do
      const int passes_left = npass - i;
      const int f = fz < left - (passes_left - 1) ? fz : left - (passes_left - 1);
      const int fr = lanes ? lane_pass_regs(lane_mode, f) : 0;
      const int q = top - f + 1;
      // the four-column passes (f <= 5, aligned) form 32-bit byte offsets
      // below 2^(q+2); the one-column passes follow column_pass_offset_bits
      const bool one_col = r.scalar_io || f > kFuseMaxFourColumn;
      const bitonic_launch_shape sh{BITONIC_LAUNCH_GLOBAL_PASS, f, q, i == 0 ? 1 : 0, 4,
                                    one_col ? column_pass_offset_bits(4, f, q) : 32};
      emit(sh, [&] {
        if (r.scalar_io)
          launch_column_pass_i32(f, i == 0, keys, n, q, st);
        else if (fr)
          (void)launch_column_lanes_pass(f, fr, i == 0, keys, n, q, st);
        else
          launch_global_pass(f, i == 0, keys, n, q, st);
      });
      top = q - 1;
    }
    const int cx = p == K ? CX_DEC : CX_NONE;
    emit(tile_shape(BITONIC_LAUNCH_TILE_MERGE, L), [&] {
      if (r.scalar_io)
        launch_tile_scalar(1, keys, n, flip, cx, st);
      else
        launch_tile(L, 1, keys, n, flip, cx, r.merge_blocks, st);
    });
  }
  return launches;
}

// The optimized kernels move keys in 16-byte vectors, which needs a 16-byte
// aligned base; other pointers take the same plan with scalar-access tile
// kernels (2^13-key tiles) and one-column passes.
static void fit_alignment(const int32_t* keys, Resolved* r) {
  if (r->kind == BITONIC_PLAN_OPTIMIZED && (reinterpret_cast<uintptr_t>(keys) & 15u) != 0) {
    r->scalar_io = true;
    r->tile = kScalarTileLog2;
    r->sort_tile = kScalarTileLog2;
  }
}

static int check_sort_args(int32_t* keys, int64_t n) {
  if (n < 0) return BITONIC_EINVAL;
  if (n > (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (n > 1 && keys == nullptr) return BITONIC_EINVAL;
  return BITONIC_OK;
}

static int finish_launches() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? BITONIC_OK : BITONIC_ELAUNCH;
}

// Per-device state: compute-unit count and the segmented sort's scratch,
// created on first use and kept until the process ends.
constexpr int kMaxDevices = 64;
struct DeviceState {
  std::atomic<int> cus{0};
};
static DeviceState g_dev[kMaxDevices];

static int current_device(int* dev) {
  if (hipGetDevice(dev) != hipSuccess || *dev < 0 || *dev >= kMaxDevices) return BITONIC_EDEVICE;
  return BITONIC_OK;
}

static int device_cus(int dev) {
  int c = g_dev[dev].cus.load(std::memory_order_relaxed);
  if (c > 0) return c;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0)
    c = 256;
  g_dev[dev].cus.store(c, std::memory_order_relaxed);
  return c;
}

// Scratch of the eager segmented sorts: one buffer per (device, stream),
// grown on demand, replaced buffers retired and never freed, the stream never
// waited for (scratch_cache.hpp).
struct HipAlloc {
  void* alloc(size_t bytes) {
    void* p = nullptr;
    return hipMalloc(&p, bytes) == hipSuccess ? p : nullptr;
  }
};
static ScratchCache<HipAlloc> g_scratch;

// An eager segmented call on a stream that is being captured into a graph
// would bind the graph to the stream's shared, growable buffer, so that its
// replays and later eager calls on other streams could race on it: such
// calls are refused (BITONIC_EINVAL).  Graphs take
// bitonic_graph_capture_segmented_i32 (a buffer of their own) or the
// allocation-free entry point.
static bool stream_is_capturing(hipStream_t st) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

static int stream_scratch(int dev, hipStream_t st, size_t bytes, void** out) {
  if (stream_is_capturing(st)) return BITONIC_EINVAL;
  void* p = g_scratch.get(dev, st, bytes);
  if (!p) return BITONIC_ENOMEM;
  *out = p;
  return BITONIC_OK;
}

// Fill in the device-dependent parts of a plan.
static int bind_device(Resolved* r) {
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  r->merge_blocks = r->merge_bpc > 0 ? (uint32_t)(device_cus(dev) * r->merge_bpc) : 0u;
  const int pb = g_phase_bpc.load();
  r->phase_blocks = pb == 0 ? r->merge_blocks : (pb > 0 ? (uint32_t)(device_cus(dev) * pb) : 0u);
  return BITONIC_OK;
}

// The big segments' tile (log2 elements) of a sort's data: 4-byte keys take
// kSegTileLog32, 8-byte elements (8-byte keys, pairs) kSegTileLog64.
static int seg_tile_log_of(const SegData& d) {
  return (d.keys64 || d.values) ? kSegTileLog64 : kSegTileLog32;
}

// The launch sequence of one segmented sort (see kernels_segmented.hip) on
// the given scratch buffer (seg_scratch_bytes(nseg) bytes); returns the
// number of launches (enqueued unless count_only; shapes to obs, with `unit`
// the bytes per element and array: 4 for 4-byte keys and pairs, 8 for 8-byte
// keys).  The kernels index segments through 64-bit pointers.
static int64_t enqueue_segmented(const SegData& d, const int64_t* offsets, int64_t nseg,
                                 int64_t max_seg_len, void* scratch, int cus, hipStream_t st,
                                 bool count_only = false, Observer* obs = nullptr,
                                 int unit = 4) {
  const int T = seg_tile_log_of(d);
  int64_t launches = 0;
  auto emit = [&](bitonic_launch_shape sh, auto&& launch) {
    if (!count_only) launch();
    if (obs && launches < obs->cap && obs->shapes) obs->shapes[launches] = sh;
    ++launches;
  };
  const SegScratch sc = count_only ? SegScratch{} : seg_scratch_carve(scratch, nseg);
  // with validation on, a check of the table comes first (one more launch,
  // not counted among the sort's launches)
  const bool validated = !count_only && validate_enabled();
  if (validated) launch_seg_validate(offsets, nseg, max_seg_len, sc, st);
  emit({BITONIC_LAUNCH_SEG_PREP, 0, 0, 0, unit, 64},
       [&] { launch_seg_prep(offsets, nseg, sc, T, validated, st); });
  const int64_t slots = (int64_t)cus * g_seg_bpc.load();
  const int small_grid = (int)(slots < nseg ? slots : nseg);
  emit({BITONIC_LAUNCH_SEG_SMALL, 0, kSegSmallMaxLog2, 0, unit, 64},
       [&] { launch_seg_small(d, offsets, sc, small_grid, st); });
  const int M = ceil_log2(max_seg_len);
  if (M <= kSegSmallMaxLog2) return launches;
  // two workgroups per CU of the 2^14-key tiles (67.6 KB of LDS each), four
  // of the 2^13-element ones
  const int grid = cus * (T == kSegTileLog32 ? 2 : 4);
  const int pass_grid = cus * g_seg_pass_bpc.load();
  emit({BITONIC_LAUNCH_TILE_SORT, 0, T, 0, unit, 64},
       [&] { launch_seg_tiles(false, d, offsets, sc, kSegSmallMaxLog2 + 1, grid, st); });
  const int fuse = g_seg_fuse.load();
  const bool phase = g_phase_merge.load() != 0;
  for (int p = T + 1; p <= M; ++p) {
    if (p == T + 1 && phase) {
      // the whole phase on units of 2^p keys (mirror step included)
      // one workgroup per CU for 4-byte keys (135 KiB of LDS), two for 8-byte
      // elements (68 KiB)
      emit({BITONIC_LAUNCH_TILE_MERGE, 0, p, 1, unit, 64},
           [&] { launch_seg_phase(d, offsets, sc, T == kSegTileLog32 ? cus : 2 * cus, st); });
      continue;
    }
    const int nb = p - T;
    const int npass = (nb + fuse - 1) / fuse;
    int top = p - 1;
    for (int i = 0; i < npass; ++i) {
      const int left = top - T + 1;
      const int f = (left + (npass - i) - 1) / (npass - i);
      const int q = top - f + 1;
      emit({BITONIC_LAUNCH_GLOBAL_PASS, f, q, i == 0 ? 1 : 0, unit, 64},
           [&] { launch_seg_pass(f, i == 0, d, offsets, sc, p, q, pass_grid, st); });
      top = q - 1;
    }
    emit({BITONIC_LAUNCH_TILE_MERGE, 0, T, 0, unit, 64},
         [&] { launch_seg_tiles(true, d, offsets, sc, p, grid, st); });
  }
  return launches;
}

}  // namespace bitonic

using namespace bitonic;

// ---------------------------------------------------------------------------
// HIP graphs

struct bitonic_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* scratch = nullptr;
};

// Capture what `enqueue` puts on a private stream into an executable graph.
template <class F>
static int capture_graph(bitonic_graph** out, void* scratch, F&& enqueue) {
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return BITONIC_EDEVICE;
  (void)hipGetLastError();
  int rc = BITONIC_OK;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = BITONIC_EDEVICE;
  } else {
    enqueue(cs);
    const hipError_t le = hipGetLastError();
    const hipError_t ce = hipStreamEndCapture(cs, &graph);
    if (le != hipSuccess) rc = BITONIC_ELAUNCH;
    else if (ce != hipSuccess || graph == nullptr) rc = BITONIC_EDEVICE;
    else if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = BITONIC_EDEVICE;
  }
  (void)hipStreamDestroy(cs);
  if (rc) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  bitonic_graph* g = new (std::nothrow) bitonic_graph;
  if (!g) {
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    return BITONIC_ENOMEM;
  }
  g->graph = graph;
  g->exec = exec;
  g->scratch = scratch;
  *out = g;
  return BITONIC_OK;
}

// The plan of the 8-byte sorts: tile sort, then for every phase p > L its
// long strides in passes of at most F steps and its last L strides in a tile
// merge -- the optimized plan of the 4-byte sort on 8-byte elements.  Returns
// the number of launches (enqueued unless count_only).
// With `unit` 4 (pairs: a 4-byte key and a 4-byte value array) or 8 (8-byte
// keys) for the shapes written to obs (bitonic_plan_shapes).
static int64_t enqueue_wide(int64_t* k64, int32_t* k32, int32_t* vals, uint32_t n, Codec64 cd,
                            int L, int F, hipStream_t st, bool count_only,
                            Observer* obs = nullptr, int unit = 8) {
  const int K = ceil_log2(n);
  if (K <= 0) return 0;
  int64_t launches = 0;
  auto emit = [&](bitonic_launch_shape sh, auto&& launch) {
    if (!count_only) launch();
    if (obs && launches < obs->cap && obs->shapes) obs->shapes[launches] = sh;
    ++launches;
  };
  auto tile_shape = [&](int kind, int Lt) { return bitonic_launch_shape{kind, 0, Lt, 0, unit, 64}; };
  if (K <= L) {
    const int Lt = K < kWideTileMinLog2 ? kWideTileMinLog2 : K;
    emit(tile_shape(BITONIC_LAUNCH_TILE_SORT, Lt),
         [&] { launch_wide_tile(Lt, 0, k64, k32, vals, n, cd, CX_BOTH, st); });
    return launches;
  }
  emit(tile_shape(BITONIC_LAUNCH_TILE_SORT, L),
       [&] { launch_wide_tile(L, 0, k64, k32, vals, n, cd, CX_ENC, st); });
  const bool phase = g_phase_merge.load() != 0;
  for (int p = L + 1; p <= K; ++p) {
    if (p == L + 1 && phase) {
      // the whole phase on 2^p-element tiles (mirror step included)
      const int cx = p == K ? CX_DEC : CX_NONE;
      emit(bitonic_launch_shape{BITONIC_LAUNCH_TILE_MERGE, 0, p, 1, unit, 64},
           [&] { launch_wide_phase(p, k64, k32, vals, n, cd, cx, st); });
      continue;
    }
    // more than kWideFuseMaxColumn steps split columns over lanes: whole
    // blocks (n a power of two) and phases up to 29 (wide_lanes_fit)
    const int Fp = (F > kWideFuseMaxColumn && ((n & (n - 1)) != 0 || p > 29)) ? kWideFuseMaxColumn : F;
    const int nb = p - L;
    const int npass = (nb + Fp - 1) / Fp;
    int top = p - 1;
    for (int i = 0; i < npass; ++i) {  // widest pass first, as for 4-byte keys
      const int left = top - L + 1;
      const int passes_left = npass - i;
      const int f = Fp < left - (passes_left - 1) ? Fp : left - (passes_left - 1);
      const int q = top - f + 1;
      const bitonic_launch_shape sh{BITONIC_LAUNCH_GLOBAL_PASS, f, q, i == 0 ? 1 : 0, unit,
                                    column_pass_offset_bits((uint32_t)unit, f, q)};
      emit(sh, [&] { launch_wide_pass(f, i == 0, k64, k32, vals, n, q, st); });
      top = q - 1;
    }
    const int cx = p == K ? CX_DEC : CX_NONE;
    emit(tile_shape(BITONIC_LAUNCH_TILE_MERGE, L),
         [&] { launch_wide_tile(L, 1, k64, k32, vals, n, cd, cx, st); });
  }
  return launches;
}

static int resolve_wide(const bitonic_plan* plan, int* L, int* F) {
  load_env_tuning_once();
  *L = g_wide_tile_log2.load();
  *F = g_wide_fuse.load();
  if (plan) {
    if (plan->kind != BITONIC_PLAN_AUTO && plan->kind != BITONIC_PLAN_OPTIMIZED)
      return BITONIC_EINVAL;
    if (plan->tile_log2) *L = plan->tile_log2;
    if (plan->fuse) *F = plan->fuse;
  }
  if (*L < kWideTileMinLog2 || *L > kWideTileMaxLog2) return BITONIC_EINVAL;
  if (*F < 1 || *F > kWideFuseMax) return BITONIC_EINVAL;
  return BITONIC_OK;
}

// Arguments of an 8-byte sort, by key_type: 8-byte keys (3..5) at keys with
// values == nullptr, or pairs of 4-byte keys (0..2) at keys and int32 values.
static int sort_wide(void* keys, int32_t* values, int64_t n, int key_type, int ascending,
                     const bitonic_plan* plan, void* stream) {
  if (key_type < BITONIC_KEY_I32 || key_type > BITONIC_KEY_F64) return BITONIC_EINVAL;
  const bool pairs = key_type <= BITONIC_KEY_F32;
  if (!pairs && values != nullptr) return BITONIC_EINVAL;
  if (n < 0) return BITONIC_EINVAL;
  if (n > (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (n > 1 && (keys == nullptr || (pairs && values == nullptr))) return BITONIC_EINVAL;
  const uintptr_t align = pairs ? 3u : 7u;
  if ((reinterpret_cast<uintptr_t>(keys) & align) != 0 ||
      (reinterpret_cast<uintptr_t>(values) & 3u) != 0)
    return BITONIC_EINVAL;
  int L = 0, F = 0;
  const int rc = resolve_wide(plan, &L, &F);
  if (rc) return rc;
  if (n <= 1) return BITONIC_OK;
  const Codec64 cd = pairs ? make_pair_codec(key_type, ascending != 0)
                           : make_codec64(key_type, ascending != 0);
  (void)hipGetLastError();
  if (pairs)
    enqueue_wide(nullptr, static_cast<int32_t*>(keys), values, (uint32_t)n, cd, L, F,
                 (hipStream_t)stream, false);
  else
    enqueue_wide(static_cast<int64_t*>(keys), nullptr, nullptr, (uint32_t)n, cd, L, F,
                 (hipStream_t)stream, false);
  return finish_launches();
}

extern "C" {

const char* bitonic_status_string(int status) {
  switch (status) {
    case BITONIC_OK: return "ok";
    case BITONIC_EINVAL: return "invalid argument";
    case BITONIC_ENOMEM: return "out of device memory";
    case BITONIC_ELAUNCH: return "kernel launch failed";
    case BITONIC_EUNSUPPORTED: return "unsupported size";
    case BITONIC_EDEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* bitonic_version(void) { return "bitonic_mi355x 0.1 (gfx950)"; }

int bitonic_sort_plan_i32(int32_t* keys, int64_t n, int ascending, const bitonic_plan* plan,
                          void* stream) {
  int rc = check_sort_args(keys, n);
  if (rc) return rc;
  Resolved r;
  rc = resolve(plan, n, &r);
  if (rc) return rc;
  if (n <= 1) return BITONIC_OK;
  fit_alignment(keys, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  (void)hipGetLastError();
  enqueue_plain(keys, (uint32_t)n, 64, make_codec(BITONIC_KEY_I32, ascending), r, (hipStream_t)stream, false);
  return finish_launches();
}

int bitonic_sort_i32(int32_t* keys, int64_t n, int ascending, void* stream) {
  return bitonic_sort_plan_i32(keys, n, ascending, nullptr, stream);
}

int bitonic_sort_keys(void* keys, int64_t n, int key_type, int ascending, void* stream) {
  if (key_type < BITONIC_KEY_I32 || key_type > BITONIC_KEY_F32) return BITONIC_EINVAL;
  int32_t* k = static_cast<int32_t*>(keys);
  int rc = check_sort_args(k, n);
  if (rc) return rc;
  Resolved r;
  rc = resolve(nullptr, n, &r);
  if (rc) return rc;
  if (n <= 1) return BITONIC_OK;
  fit_alignment(k, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  (void)hipGetLastError();
  enqueue_plain(k, (uint32_t)n, 64, make_codec(key_type, ascending != 0), r, (hipStream_t)stream,
                false);
  return finish_launches();
}

int bitonic_network_phases_i32(int32_t* keys, int64_t n, int ascending, int last_phase,
                               const bitonic_plan* plan, void* stream) {
  int rc = check_sort_args(keys, n);
  if (rc) return rc;
  if (last_phase < 1) return BITONIC_EINVAL;
  Resolved r;
  rc = resolve(plan, n, &r);
  if (rc) return rc;
  if (n <= 1) return BITONIC_OK;
  fit_alignment(keys, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  (void)hipGetLastError();
  enqueue_plain(keys, (uint32_t)n, last_phase, make_codec(BITONIC_KEY_I32, ascending), r, (hipStream_t)stream, false);
  return finish_launches();
}

int bitonic_sort_keys64(void* keys, int64_t n, int key_type, int ascending, void* stream) {
  if (key_type < BITONIC_KEY_I64 || key_type > BITONIC_KEY_F64) return BITONIC_EINVAL;
  return sort_wide(keys, nullptr, n, key_type, ascending, nullptr, stream);
}

int bitonic_sort_pairs(void* keys, int32_t* values, int64_t n, int key_type, int ascending,
                       void* stream) {
  if (key_type < BITONIC_KEY_I32 || key_type > BITONIC_KEY_F32) return BITONIC_EINVAL;
  return sort_wide(keys, values, n, key_type, ascending, nullptr, stream);
}

int bitonic_sort_wide_plan(void* keys, int32_t* values, int64_t n, int key_type, int ascending,
                           const bitonic_plan* plan, void* stream) {
  return sort_wide(keys, values, n, key_type, ascending, plan, stream);
}

int64_t bitonic_wide_plan_passes(int64_t n, const bitonic_plan* plan) {
  if (n < 0 || n > (int64_t(1) << 31)) return -1;
  int L = 0, F = 0;
  if (resolve_wide(plan, &L, &F)) return -1;
  if (n <= 1) return 0;
  return enqueue_wide(nullptr, nullptr, nullptr, (uint32_t)n, Codec64{0, 0}, L, F, nullptr, true);
}

int bitonic_plan_tile_log2(int64_t n, const bitonic_plan* plan) {
  if (n < 0 || n > (int64_t(1) << 31)) return -1;
  Resolved r;
  if (resolve(plan, n, &r)) return -1;
  return r.kind == BITONIC_PLAN_BASIC ? 0 : r.tile;
}

int64_t bitonic_plan_passes(int64_t n, const bitonic_plan* plan) {
  if (n < 0 || n > (int64_t(1) << 31)) return -1;
  Resolved r;
  if (resolve(plan, n, &r)) return -1;
  if (n <= 1) return 0;
  return enqueue_plain(nullptr, (uint32_t)n, 64, Codec{0, 0}, r, nullptr, true);
}

int64_t bitonic_plan_describe(int64_t n, const bitonic_plan* plan, int32_t* kinds,
                              int32_t* fuse, int64_t cap) {
  if (n < 0 || n > (int64_t(1) << 31) || cap < 0) return -1;
  Resolved r;
  if (resolve(plan, n, &r)) return -1;
  if (n <= 1) return 0;
  Observer obs;
  obs.kinds = kinds;
  obs.fuse = fuse;
  obs.cap = cap;
  return enqueue_plain(nullptr, (uint32_t)n, 64, Codec{0, 0}, r, nullptr, true, &obs);
}

int64_t bitonic_plan_shapes(int64_t n, int layout, const bitonic_plan* plan,
                            bitonic_launch_shape* shapes, int64_t cap) {
  if (n < 0 || n > (int64_t(1) << 31) || cap < 0) return -1;
  Observer obs;
  obs.shapes = shapes;
  obs.cap = shapes ? cap : 0;
  switch (layout) {
    case BITONIC_LAYOUT_KEYS32:
    case BITONIC_LAYOUT_KEYS32_UNALIGNED: {
      Resolved r;
      if (resolve(plan, n, &r)) return -1;
      if (n <= 1) return 0;
      if (layout == BITONIC_LAYOUT_KEYS32_UNALIGNED)
        fit_alignment(reinterpret_cast<const int32_t*>(uintptr_t(4)), &r);
      return enqueue_plain(nullptr, (uint32_t)n, 64, Codec{0, 0}, r, nullptr, true, &obs);
    }
    case BITONIC_LAYOUT_KEYS64:
    case BITONIC_LAYOUT_PAIRS: {
      int L = 0, F = 0;
      if (resolve_wide(plan, &L, &F)) return -1;
      if (n <= 1) return 0;
      return enqueue_wide(nullptr, nullptr, nullptr, (uint32_t)n, Codec64{0, 0}, L, F, nullptr,
                          true, &obs, layout == BITONIC_LAYOUT_KEYS64 ? 8 : 4);
    }
    case BITONIC_LAYOUT_SEG_KEYS32:
    case BITONIC_LAYOUT_SEG_PAIRS:
    case BITONIC_LAYOUT_SEG_KEYS64: {
      if (n == 0) return 0;
      SegData d{};  // only which storage it is matters when counting
      int32_t dummy32 = 0;
      int64_t dummy64 = 0;
      if (layout == BITONIC_LAYOUT_SEG_PAIRS) d.values = &dummy32;
      if (layout == BITONIC_LAYOUT_SEG_KEYS64) d.keys64 = &dummy64;
      return enqueue_segmented(d, nullptr, 1, n, nullptr, 256, nullptr, true, &obs,
                               layout == BITONIC_LAYOUT_SEG_KEYS64 ? 8 : 4);
    }
    default:
      return -1;
  }
}

int bitonic_sort_plan_events_i32(int32_t* keys, int64_t n, int ascending,
                                 const bitonic_plan* plan, void** events, int64_t nevents,
                                 void* stream) {
  int rc = check_sort_args(keys, n);
  if (rc) return rc;
  if (nevents < 0 || (nevents > 0 && events == nullptr)) return BITONIC_EINVAL;
  Resolved r;
  rc = resolve(plan, n, &r);
  if (rc) return rc;
  if (n <= 1) return BITONIC_OK;
  fit_alignment(keys, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  Observer obs;
  obs.events = reinterpret_cast<hipEvent_t*>(events);
  obs.nevents = nevents;
  (void)hipGetLastError();
  enqueue_plain(keys, (uint32_t)n, 64, make_codec(BITONIC_KEY_I32, ascending), r, (hipStream_t)stream, false, &obs);
  return finish_launches();
}

int bitonic_sort_plan_launches_i32(int32_t* keys, int64_t n, int ascending,
                                   const bitonic_plan* plan, int64_t first, int64_t count,
                                   void* stream) {
  int rc = check_sort_args(keys, n);
  if (rc) return rc;
  if (first < 0 || count < 0) return BITONIC_EINVAL;
  Resolved r;
  rc = resolve(plan, n, &r);
  if (rc) return rc;
  if (n <= 1 || count == 0) return BITONIC_OK;
  fit_alignment(keys, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  Observer obs;
  obs.first = first;
  obs.count = count;
  (void)hipGetLastError();
  enqueue_plain(keys, (uint32_t)n, 64, make_codec(BITONIC_KEY_I32, ascending), r, (hipStream_t)stream, false, &obs);
  return finish_launches();
}

int bitonic_sort_segmented_bounded_i32(int32_t* keys, const int64_t* offsets, int64_t nseg,
                                       int64_t max_seg_len, int ascending, void* stream) {
  return bitonic_sort_segmented_keys(keys, offsets, nseg, max_seg_len, BITONIC_KEY_I32, ascending,
                                     stream);
}

// A bound on the segment length when the caller gives none, found without
// reading the offsets: no segment reaches past the end of the device
// allocation that holds the keys (hipMemGetAddressRange consults the
// runtime's allocation records on the host; nothing is enqueued or waited
// for).  Where the range is unknown the bound is 2^31.  The phases between the
// longest segment present and this bound find no segment of their class on
// the device and return at once.
static int64_t allocation_bound(const void* keys, int elem_bytes) {
  const int64_t cap = int64_t(1) << 31;
  void* base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(keys)) != hipSuccess || !base) {
    (void)hipGetLastError();
    return cap;
  }
  const uintptr_t end = reinterpret_cast<uintptr_t>(base) + size;
  const uintptr_t at = reinterpret_cast<uintptr_t>(keys);
  if (end <= at) return cap;
  const int64_t elems = (int64_t)((end - at) / (uintptr_t)elem_bytes);
  return elems < 1 ? 1 : (elems < cap ? elems : cap);
}

// Segmented sort of keys of any key type (values == nullptr) or of (key,
// value) pairs with 4-byte keys.
static int sort_segmented(void* keys_v, int32_t* values, const int64_t* offsets, int64_t nseg,
                          int64_t max_seg_len, int key_type, int ascending, void* stream) {
  int32_t* keys = static_cast<int32_t*>(keys_v);
  if (key_type < BITONIC_KEY_I32 || key_type > BITONIC_KEY_F64) return BITONIC_EINVAL;
  const bool wide_keys = key_type >= BITONIC_KEY_I64;
  if (wide_keys && values != nullptr) return BITONIC_EINVAL;
  if (nseg < 0 || max_seg_len < 0) return BITONIC_EINVAL;
  if (nseg >= (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (max_seg_len > (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (nseg == 0) return BITONIC_OK;
  if (keys == nullptr || offsets == nullptr) return BITONIC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(keys) & (wide_keys ? 7u : 3u)) != 0 ||
      (reinterpret_cast<uintptr_t>(values) & 3u) != 0)
    return BITONIC_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  load_env_tuning_once();
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  if (max_seg_len == 0) max_seg_len = allocation_bound(keys_v, wide_keys ? 8 : 4);
  void* base = nullptr;
  rc = stream_scratch(dev, st, seg_scratch_bytes(nseg), &base);
  if (rc) return rc;
  (void)hipGetLastError();
  SegData d{};
  if (wide_keys) {
    d.keys64 = static_cast<int64_t*>(keys_v);
    d.cd64 = make_codec64(key_type, ascending != 0);
  } else {
    d.keys = keys;
    d.values = values;
    d.cd = make_codec(key_type, ascending != 0);
    d.cd64 = make_pair_codec(key_type, ascending != 0);
  }
  enqueue_segmented(d, offsets, nseg, max_seg_len, base, device_cus(dev), st);
  return finish_launches();
}

int bitonic_sort_segmented_keys(void* keys, const int64_t* offsets, int64_t nseg,
                                int64_t max_seg_len, int key_type, int ascending, void* stream) {
  return sort_segmented(keys, nullptr, offsets, nseg, max_seg_len, key_type, ascending, stream);
}

int bitonic_sort_segmented_pairs(void* keys, int32_t* values, const int64_t* offsets,
                                 int64_t nseg, int64_t max_seg_len, int key_type, int ascending,
                                 void* stream) {
  if (key_type < BITONIC_KEY_I32 || key_type > BITONIC_KEY_F32) return BITONIC_EINVAL;
  if (nseg > 0 && values == nullptr) return BITONIC_EINVAL;
  return sort_segmented(keys, values, offsets, nseg, max_seg_len, key_type, ascending, stream);
}

int bitonic_validation_error(int32_t* code) {
  if (!code) return BITONIC_EINVAL;
  return seg_validation_error(code) == 0 ? BITONIC_OK : BITONIC_EDEVICE;
}

int64_t bitonic_segmented_default_bound(const void* keys, int key_bytes) {
  if (keys == nullptr || (key_bytes != 4 && key_bytes != 8)) return -1;
  return allocation_bound(keys, key_bytes);
}

int bitonic_sort_segmented_noalloc_i32(int32_t* keys, const int64_t* offsets, int64_t nseg,
                                       int64_t max_seg_len, int ascending, void* stream) {
  if (nseg < 0 || max_seg_len < 0) return BITONIC_EINVAL;
  if (nseg > kNoAllocMaxSegments || max_seg_len > (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (nseg == 0) return BITONIC_OK;
  if (max_seg_len < 1 || keys == nullptr || offsets == nullptr) return BITONIC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(keys) & 3u) != 0) return BITONIC_EINVAL;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  void* base = nullptr;
  if (noalloc_scratch(dev, &base) != 0) return BITONIC_EDEVICE;
  (void)hipGetLastError();
  SegData d{};
  d.keys = keys;
  d.cd = make_codec(BITONIC_KEY_I32, ascending != 0);
  d.cd64 = make_pair_codec(BITONIC_KEY_I32, ascending != 0);
  enqueue_segmented(d, offsets, nseg, max_seg_len, base, device_cus(dev), (hipStream_t)stream);
  return finish_launches();
}

int bitonic_sort_segmented_i32(int32_t* keys, const int64_t* offsets, int64_t nseg,
                               int ascending, void* stream) {
  return bitonic_sort_segmented_bounded_i32(keys, offsets, nseg, 0, ascending, stream);
}

int bitonic_set_tuning(int tile_log2, int fuse, int merge_blocks_per_cu) {
  if (tile_log2 && !tile_log2_supported(tile_log2)) return BITONIC_EINVAL;
  if (fuse && (fuse < 1 || fuse > kFuseMax)) return BITONIC_EINVAL;
  if (merge_blocks_per_cu < -1 || merge_blocks_per_cu > 16) return BITONIC_EINVAL;
  if (tile_log2) g_tile_log2.store(tile_log2);
  if (fuse) g_fuse.store(fuse);
  if (merge_blocks_per_cu > 0) g_merge_bpc.store(merge_blocks_per_cu);
  if (merge_blocks_per_cu < 0) g_merge_bpc.store(0);
  return BITONIC_OK;
}

// "name@k": an entry of size bucket k (0..31) for tile_log2, fuse or
// merge_blocks_per_cu; 0 removes it.
static int set_bucket_value(const char* name, size_t len, int k, int value) {
  if (k < 0 || k >= kBuckets) return BITONIC_EINVAL;
  auto is = [&](const char* s) { return std::strlen(s) == len && !std::strncmp(name, s, len); };
  if (is("tile_log2")) {
    if (value && !tile_log2_supported(value)) return BITONIC_EINVAL;
    g_bk_tile[k].store(value);
  } else if (is("fuse")) {
    if (value && (value < 1 || value > kFuseMax)) return BITONIC_EINVAL;
    g_bk_fuse[k].store(value);
  } else if (is("merge_blocks_per_cu")) {
    if (value < -1 || value > 16) return BITONIC_EINVAL;
    g_bk_merge[k].store(value);
  } else if (is("lane_pass")) {
    if (value != 0 && value != 7 && value != 8 && value != 9) return BITONIC_EINVAL;
    g_bk_lane[k].store(value);
  } else if (is("sort_tile_log2")) {
    if (value && !tile_log2_supported(value)) return BITONIC_EINVAL;
    g_bk_sort_tile[k].store(value);
  } else {
    return BITONIC_EINVAL;
  }
  return BITONIC_OK;
}

static bool parse_bucket_key(const char* key, size_t* len, int* k) {
  const char* at = std::strchr(key, '@');
  if (!at || !at[1]) return false;
  char* end = nullptr;
  const long v = std::strtol(at + 1, &end, 10);
  if (*end != 0 || v < 0 || v >= kBuckets) {
    *k = -1;
  } else {
    *k = (int)v;
  }
  *len = (size_t)(at - key);
  return true;
}

int bitonic_set_tuning_value(const char* key, int value) {
  if (!key) return BITONIC_EINVAL;
  {
    size_t len = 0;
    int k = 0;
    if (parse_bucket_key(key, &len, &k)) return set_bucket_value(key, len, k, value);
  }
  if (!std::strcmp(key, "tile_log2")) {
    if (value == 0) {  // back to the library's choice by n
      g_tile_log2.store(0);
      return BITONIC_OK;
    }
    return bitonic_set_tuning(value, 0, 0);
  }
  if (!std::strcmp(key, "fuse")) return value ? bitonic_set_tuning(0, value, 0) : BITONIC_EINVAL;
  if (!std::strcmp(key, "merge_blocks_per_cu"))
    return value ? bitonic_set_tuning(0, 0, value) : BITONIC_EINVAL;
  if (!std::strcmp(key, "seg_blocks_per_cu")) {
    if (value < 1 || value > 16) return BITONIC_EINVAL;
    g_seg_bpc.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "seg_pass_blocks_per_cu")) {
    if (value < 1 || value > 32) return BITONIC_EINVAL;
    g_seg_pass_bpc.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "seg_fuse")) {
    if (value < 1 || value > kSegFuseMax) return BITONIC_EINVAL;
    g_seg_fuse.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "validate")) {
    if (value < 0 || value > 1) return BITONIC_EINVAL;
    g_validate.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "tile_lane_steps")) {
    if (value < 0 || value > 1) return BITONIC_EINVAL;
    g_tile_lane.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "phase_blocks_per_cu")) {
    if (value < -1 || value > 16) return BITONIC_EINVAL;
    g_phase_bpc.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "phase_merge")) {
    if (value < 0 || value > 1) return BITONIC_EINVAL;
    g_phase_merge.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "lane_pass")) {
    if (value != 0 && value != 7 && value != 8 && value != 9) return BITONIC_EINVAL;
    g_lane_pass.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "sort_tile_log2")) {
    if (value && !tile_log2_supported(value)) return BITONIC_EINVAL;
    g_sort_tile.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "wide_tile_log2")) {
    if (value < kWideTileMinLog2 || value > kWideTileMaxLog2) return BITONIC_EINVAL;
    g_wide_tile_log2.store(value);
    return BITONIC_OK;
  }
  if (!std::strcmp(key, "wide_fuse")) {
    if (value < 1 || value > kWideFuseMax) return BITONIC_EINVAL;
    g_wide_fuse.store(value);
    return BITONIC_OK;
  }
  return BITONIC_EINVAL;
}

int bitonic_get_tuning_value(const char* key, int* value) {
  if (!key || !value) return BITONIC_EINVAL;
  {
    size_t len = 0;
    int k = 0;
    if (parse_bucket_key(key, &len, &k)) {
      if (k < 0) return BITONIC_EINVAL;
      auto is = [&](const char* s) { return std::strlen(s) == len && !std::strncmp(key, s, len); };
      if (is("tile_log2")) *value = g_bk_tile[k].load();
      else if (is("fuse")) *value = g_bk_fuse[k].load();
      else if (is("merge_blocks_per_cu")) *value = g_bk_merge[k].load();
      else if (is("lane_pass")) *value = g_bk_lane[k].load();
      else if (is("sort_tile_log2")) *value = g_bk_sort_tile[k].load();
      else return BITONIC_EINVAL;
      return BITONIC_OK;
    }
  }
  if (!std::strcmp(key, "tile_log2")) *value = g_tile_log2.load();
  else if (!std::strcmp(key, "fuse")) *value = g_fuse.load();
  else if (!std::strcmp(key, "merge_blocks_per_cu")) *value = g_merge_bpc.load() ? g_merge_bpc.load() : -1;
  else if (!std::strcmp(key, "seg_blocks_per_cu")) *value = g_seg_bpc.load();
  else if (!std::strcmp(key, "seg_pass_blocks_per_cu")) *value = g_seg_pass_bpc.load();
  else if (!std::strcmp(key, "seg_fuse")) *value = g_seg_fuse.load();
  else if (!std::strcmp(key, "tile_lane_steps")) *value = g_tile_lane.load();
  else if (!std::strcmp(key, "lane_pass")) *value = g_lane_pass.load();
  else if (!std::strcmp(key, "sort_tile_log2")) *value = g_sort_tile.load();
  else if (!std::strcmp(key, "phase_merge")) *value = g_phase_merge.load();
  else if (!std::strcmp(key, "phase_blocks_per_cu")) *value = g_phase_bpc.load();
  else if (!std::strcmp(key, "validate")) *value = validate_enabled() ? 1 : 0;
  else if (!std::strcmp(key, "wide_tile_log2")) *value = g_wide_tile_log2.load();
  else if (!std::strcmp(key, "wide_fuse")) *value = g_wide_fuse.load();
  else return BITONIC_EINVAL;
  return BITONIC_OK;
}

int bitonic_load_tuning(const char* path) {
  if (!path) return BITONIC_EINVAL;
  FILE* f = std::fopen(path, "r");
  if (!f) return BITONIC_EINVAL;
  // "<name> <value>" lines; '#' starts a comment.  A "cus <count>" line ties
  // the file to devices with that many compute units: on another device
  // nothing in the file is applied.
  struct Entry {
    char key[64];
    int value;
  };
  std::vector<Entry> entries;
  char line[256];
  int rc = BITONIC_OK;
  int cus = 0;
  while (std::fgets(line, sizeof line, f)) {
    char* hash = std::strchr(line, '#');
    if (hash) *hash = 0;
    Entry e{};
    char extra[8];
    const int got = std::sscanf(line, "%63s %d %7s", e.key, &e.value, extra);
    if (got <= 0) continue;  // blank or comment
    if (got != 2) {
      rc = BITONIC_EINVAL;
      continue;
    }
    if (!std::strcmp(e.key, "cus")) cus = e.value;
    else entries.push_back(e);
  }
  std::fclose(f);
  if (cus > 0) {
    int dev = 0, have = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&have, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        have > 0 && have != cus)
      return BITONIC_EUNSUPPORTED;
    (void)hipGetLastError();
  }
  for (const Entry& e : entries) {
    const int r = bitonic_set_tuning_value(e.key, e.value);
    if (r) rc = r;
  }
  return rc;
}

int bitonic_graph_capture_sort_i32(bitonic_graph** out, int32_t* keys, int64_t n, int ascending,
                                   const bitonic_plan* plan) {
  if (!out) return BITONIC_EINVAL;
  *out = nullptr;
  int rc = check_sort_args(keys, n);
  if (rc) return rc;
  Resolved r;
  rc = resolve(plan, n, &r);
  if (rc) return rc;
  fit_alignment(keys, &r);
  rc = bind_device(&r);
  if (rc) return rc;
  return capture_graph(out, nullptr, [&](hipStream_t cs) {
    if (n > 1) enqueue_plain(keys, (uint32_t)n, 64, make_codec(BITONIC_KEY_I32, ascending), r, cs, false);
  });
}

int bitonic_graph_capture_segmented_i32(bitonic_graph** out, int32_t* keys,
                                        const int64_t* offsets, int64_t nseg,
                                        int64_t max_seg_len, int ascending) {
  if (!out) return BITONIC_EINVAL;
  *out = nullptr;
  if (nseg < 0 || max_seg_len < 1) return BITONIC_EINVAL;
  if (nseg >= (int64_t(1) << 31) || max_seg_len > (int64_t(1) << 31)) return BITONIC_EUNSUPPORTED;
  if (nseg > 0 && (keys == nullptr || offsets == nullptr)) return BITONIC_EINVAL;
  int dev = 0;
  int rc = current_device(&dev);
  if (rc) return rc;
  void* scratch = nullptr;
  if (nseg > 0 && hipMalloc(&scratch, seg_scratch_bytes(nseg)) != hipSuccess) return BITONIC_ENOMEM;
  const int cus = device_cus(dev);
  rc = capture_graph(out, scratch, [&](hipStream_t cs) {
    if (nseg > 0) {
      SegData d{};
      d.keys = keys;
      d.cd = make_codec(BITONIC_KEY_I32, ascending != 0);
      enqueue_segmented(d, offsets, nseg, max_seg_len, scratch, cus, cs);
    }
  });
  if (rc && scratch) (void)hipFree(scratch);
  return rc;
}

int bitonic_graph_launch(bitonic_graph* g, void* stream) {
  if (!g || !g->exec) return BITONIC_EINVAL;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? BITONIC_OK : BITONIC_ELAUNCH;
}

int bitonic_graph_destroy(bitonic_graph* g) {
  if (!g) return BITONIC_OK;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->scratch) (void)hipFree(g->scratch);
  delete g;
  return BITONIC_OK;
}

int bitonic_keygen_i32(int32_t* out, int64_t n, uint64_t seed, int64_t start, void* stream) {
  if (n < 0 || start < 0 || (n > 0 && out == nullptr)) return BITONIC_EINVAL;
  if (n == 0) return BITONIC_OK;
  (void)hipGetLastError();
  launch_keygen(out, (uint64_t)n, seed, (uint64_t)start, (hipStream_t)stream);
  return finish_launches();
}

}  // extern "C"
