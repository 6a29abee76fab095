/*
 * bitonic.h -- C interface of the MI355X (gfx950) bitonic sort library
 * (libbitonic_mi355x.so).
 *
 * The library sorts 32-bit signed integer keys on one GPU with the bitonic
 * sorting network of Mu, Cui and Song, "The implementation and optimization
 * of Bitonic sort algorithm based on CUDA" (arXiv 1506.01446): for
 * N = 2^k keys the network has k phases, phase r merges blocks of 2^r keys
 * in r compare-exchange steps, k(k+1)/2 steps in all (sections 3.1-3.3).
 * Steps whose comparators stay inside one on-chip tile run in LDS and
 * registers (the paper's optimization 1, section 4.1); consecutive steps
 * with longer strides are fused into one pass over HBM with the keys held in
 * registers (optimization 2, section 4.2).
 *
 * Conventions shared by every entry point:
 *  - Key and offset pointers are DEVICE pointers (hipMalloc or torch CUDA
 *    tensors); the caller owns them.  Sorting is in place.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls are
 *    asynchronous: they enqueue kernels on `stream` and return; the keys are
 *    sorted once the stream reaches that point.  The host never blocks.
 *  - Keys compare as signed int32.  `ascending` != 0 sorts ascending,
 *    0 descending.  The result is unique (keys only), so it is bit-exact
 *    whatever the plan.
 *  - n that is not a power of two is handled as if padded to N = 2^k with
 *    INT32_MAX sentinels (section 3 assumes n = 2^k).  The sentinels are
 *    never stored: the network is run in its "flip" arrangement (first step
 *    of each phase compares mirror images, every comparator puts the smaller
 *    key at the lower index), in which a comparator whose upper end is a
 *    sentinel never moves anything, so it is skipped.
 *  - The optimized kernels move keys in 16-byte vectors; a keys pointer that
 *    is not 16-byte aligned (but 4-byte aligned) is sorted by the same plan
 *    with scalar-access tile kernels of 2^13 keys and one-column passes
 *    (same result).
 *  - Errors in the arguments are reported synchronously and nothing is
 *    enqueued.  No exception crosses this interface.
 *  - Calls are reentrant on different streams.  The eager segmented sorts
 *    use a scratch buffer per (device, stream) that the library allocates on
 *    first use on that stream, and replaces by a larger one when a call needs
 *    more; a replaced buffer is kept (never freed) until the process ends,
 *    since work enqueued earlier may still use it, so no call waits for the
 *    stream.  Segmented calls on one stream are ordered by the stream, calls
 *    on different streams use different buffers.
 */
#ifndef BITONIC_MI355X_H
#define BITONIC_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum bitonic_status {
  BITONIC_OK = 0,
  BITONIC_EINVAL = -1,       /* bad argument (null pointer, negative size, bad plan) */
  BITONIC_ENOMEM = -2,       /* scratch allocation failed */
  BITONIC_ELAUNCH = -3,      /* a kernel launch failed (hipGetLastError) */
  BITONIC_EUNSUPPORTED = -4, /* size beyond what the library handles (n > 2^31) */
  BITONIC_EDEVICE = -5       /* no usable gfx950 device / HIP runtime error */
};

/* Text for a status code (static storage, never NULL). */
const char* bitonic_status_string(int status);

/*
 * Sort keys[0, n) in place (sections 3.1-3.3, 4.1, 4.2).
 *   keys       device pointer to n int32 keys (may be NULL when n <= 1)
 *   n          number of keys, 0 <= n <= 2^31; n <= 1 enqueues nothing
 *   ascending  nonzero: ascending; zero: descending
 *   stream     hipStream_t to enqueue on
 * Returns BITONIC_OK, BITONIC_EINVAL (keys NULL with n > 1, n < 0),
 * BITONIC_EUNSUPPORTED (n > 2^31) or BITONIC_ELAUNCH.
 */
int bitonic_sort_i32(int32_t* keys, int64_t n, int ascending, void* stream);

/*
 * Key types.  Every type is sorted with the same network; a key type only
 * changes the order-preserving map applied as keys are loaded and stored
 * (the paper's future work, section 6, names other key types):
 *   BITONIC_KEY_I32  signed two's-complement integers
 *   BITONIC_KEY_U32  unsigned integers
 *   BITONIC_KEY_F32  IEEE-754 binary32, in the totalOrder of IEEE 754-2008
 *                    (-NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN; NaNs
 *                    ordered by their payload bits)
 *   BITONIC_KEY_I64, BITONIC_KEY_U64, BITONIC_KEY_F64  the same on 8 bytes
 *                    (binary64 for F64)
 */
enum bitonic_key_type {
  BITONIC_KEY_I32 = 0,
  BITONIC_KEY_U32 = 1,
  BITONIC_KEY_F32 = 2,
  BITONIC_KEY_I64 = 3,
  BITONIC_KEY_U64 = 4,
  BITONIC_KEY_F64 = 5
};

/*
 * bitonic_sort_i32 for any key type (keys: device pointer to n 4-byte keys
 * of that type).  Returns BITONIC_EINVAL for an unknown key_type, else as
 * bitonic_sort_i32.
 */
int bitonic_sort_keys(void* keys, int64_t n, int key_type, int ascending, void* stream);

/*
 * Sort n 8-byte keys in place: the network of sections 3.1-3.3 with the
 * tile sort and fused passes of sections 4.1-4.2 on 8-byte elements.
 *   keys       device pointer to n keys of key_type (BITONIC_KEY_I64, U64
 *              or F64), 8-byte aligned (may be NULL when n <= 1)
 *   n, ascending, stream  as for bitonic_sort_i32
 * Returns BITONIC_EINVAL for another key_type, a misaligned pointer, keys
 * NULL with n > 1 or n < 0; else as bitonic_sort_i32.
 */
int bitonic_sort_keys64(void* keys, int64_t n, int key_type, int ascending, void* stream);

/*
 * Sort (key, value) pairs in place by key, ties by value: a key-value
 * variant of the same network, each pair moving through it as one 8-byte
 * element (key word, then value word).  The result is the unique order of
 * the pairs by key in the requested direction (key_type BITONIC_KEY_I32,
 * U32 or F32, as for bitonic_sort_keys) and, among equal keys, by value
 * ascending as int32.  With values 0 .. n-1 on input, the values come out as
 * the permutation of a stable sort (an argsort).
 *   keys       device pointer to n 4-byte keys, 4-byte aligned
 *   values     device pointer to n int32 values, 4-byte aligned (both may
 *              be NULL when n <= 1; the arrays must not overlap)
 *   n, ascending, stream  as for bitonic_sort_i32
 * Returns as bitonic_sort_keys64.
 */
int bitonic_sort_pairs(void* keys, int32_t* values, int64_t n, int key_type, int ascending,
                       void* stream);

/*
 * Sort every segment of a CSR table independently, in one batched launch
 * sequence (the network of section 3 applied per segment, each segment
 * padded virtually to its own power of two).
 *   keys       device pointer; segment s is keys[offsets[s], offsets[s+1])
 *   offsets    DEVICE pointer to nseg + 1 nondecreasing int64 offsets
 *              (offsets[0] need not be 0; empty segments are allowed;
 *              segments must not overlap and each must hold < 2^31 keys)
 *   nseg       number of segments, >= 0; 0 enqueues nothing
 *   ascending  as above, for every segment
 *   stream     hipStream_t
 * The call only enqueues work; it never reads the offsets on the host and
 * never waits.  How many merge phases it enqueues depends on a bound on the
 * segment length: here the number of keys from `keys` to the end of the
 * device allocation that holds them (the runtime's allocation records,
 * consulted on the host), or 2^31 where that is unknown.  Phases past the
 * longest segment actually present find no segment of their class on the
 * device and return at once, at the cost of their launches (a few
 * microseconds each); bitonic_sort_segmented_bounded_i32 with a tight bound
 * enqueues only the phases needed.  Bad offsets are undefined behaviour
 * unless offsets validation is on (bitonic_validation_error).
 * Calls on a stream that is being captured into a graph are refused
 * (BITONIC_EINVAL): the graph would share the stream's scratch buffer with
 * later eager calls; capture bitonic_graph_capture_segmented_i32 or
 * bitonic_sort_segmented_noalloc_i32 instead.
 * Returns BITONIC_OK, BITONIC_EINVAL, BITONIC_ENOMEM (scratch), BITONIC_EDEVICE
 * or BITONIC_ELAUNCH.
 */
int bitonic_sort_segmented_i32(int32_t* keys, const int64_t* offsets,
                               int64_t nseg, int ascending, void* stream);

/*
 * Offsets validation (for debugging; off by default).  With the tuning value
 * "validate" set to 1, or else the environment variable BITONIC_VALIDATE=1,
 * every segmented sort first checks its offsets table on the device: offsets
 * nondecreasing, offsets[0] >= 0, every segment below 2^31 keys and at most
 * the bound (max_seg_len, or the default bound).  A table that fails is not
 * sorted (the keys are left as they were) and its error is recorded on the
 * device.  bitonic_validation_error waits for the device to be idle, then
 * writes the first error recorded since its last call (0 none, 1 decreasing
 * offsets, 2 a segment of 2^31 keys or more, 3 a segment longer than the
 * bound, 4 offsets[0] < 0) to *code and clears it.  Without validation, bad
 * offsets are undefined behaviour.  Returns BITONIC_OK, BITONIC_EINVAL (code
 * NULL) or BITONIC_EDEVICE.
 */
int bitonic_validation_error(int32_t* code);

/*
 * The bound on the segment length that the segmented sorts take when the
 * caller gives none (max_seg_len 0): the number of key_bytes-byte keys (4 or
 * 8) from `keys` to the end of the device allocation holding them, at most
 * 2^31 (2^31 where the allocation is unknown).  Host-side; nothing is
 * enqueued.  -1 for a NULL pointer or another key size.  The merge phases
 * enqueued are those up to ceil(log2 bound) (bitonic_plan_shapes with a
 * segmented layout and n = bound lists the launches).
 */
int64_t bitonic_segmented_default_bound(const void* keys, int key_bytes);

/*
 * As bitonic_sort_segmented_i32, with a host-side bound: every segment holds
 * at most max_seg_len keys (0 = unknown: then the bound of
 * bitonic_sort_segmented_i32 is taken).  The bound fixes how many merge
 * phases are enqueued; a segment longer than the bound is undefined
 * behaviour.  Launches: a prep kernel, one persistent kernel for all segments
 * of up to 2^13 keys, and, if the bound exceeds 2^13, one tile-sort launch
 * plus, per phase p = 14 .. ceil(log2 bound), its fused long-stride passes
 * (at most "seg_fuse" steps each, default 5) and one tile merge.  Like
 * bitonic_sort_segmented_i32 it refuses a capturing stream.
 */
int bitonic_sort_segmented_bounded_i32(int32_t* keys, const int64_t* offsets,
                                       int64_t nseg, int64_t max_seg_len,
                                       int ascending, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc): the segmented sort
 * of bitonic_sort_segmented_bounded_i32 with the same launch sequence and
 * kernels, whose scratch (the segment classification and prefix tables) is a
 * file-scope device array of 6 MiB + 1 KiB that each GPU the library runs on
 * holds until the process ends.  The call allocates and frees nothing, never
 * blocks, and may be captured into a HIP graph.
 *   keys, offsets, ascending, stream  as for bitonic_sort_segmented_bounded_i32
 *   nseg         0 <= nseg <= 262143 (2^18 - 1); larger tables return
 *                BITONIC_EUNSUPPORTED with nothing enqueued
 *   max_seg_len  bound on the segment length, 1 .. 2^31, required when
 *                nseg > 0 (BITONIC_EINVAL otherwise)
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (each call's first kernel rewrites what it reads): calls
 * that overlap on one GPU (on different streams, or replays of captured
 * graphs that are not ordered with each other or with eager calls) race and
 * give undefined results; calls ordered on one stream do not.
 * Returns BITONIC_OK, BITONIC_EINVAL, BITONIC_EUNSUPPORTED, BITONIC_EDEVICE
 * (the array's address could not be taken) or BITONIC_ELAUNCH.
 */
int bitonic_sort_segmented_noalloc_i32(int32_t* keys, const int64_t* offsets,
                                       int64_t nseg, int64_t max_seg_len,
                                       int ascending, void* stream);

/* bitonic_sort_segmented_bounded_i32 for any key type (max_seg_len 0 =
 * unknown, as above): 4-byte keys need 4-byte alignment, 8-byte keys
 * (BITONIC_KEY_I64, U64, F64) 8-byte alignment; BITONIC_EINVAL for an
 * unknown key_type or a misaligned pointer. */
int bitonic_sort_segmented_keys(void* keys, const int64_t* offsets, int64_t nseg,
                                int64_t max_seg_len, int key_type, int ascending,
                                void* stream);

/*
 * Segmented sort of (key, value) pairs: every segment of the CSR table is
 * sorted as bitonic_sort_pairs sorts one array (by key in the requested
 * direction, equal keys by value ascending as int32; with values 0..len-1 per
 * segment, a stable per-segment argsort), in the batched launch sequence of
 * bitonic_sort_segmented_i32 on 8-byte elements.
 *   keys, values  device pointers to the 4-byte keys (key_type
 *                 BITONIC_KEY_I32, U32 or F32) and the int32 values, both
 *                 indexed by the offsets, 4-byte aligned, not overlapping
 *   offsets, nseg, max_seg_len, ascending, stream  as for
 *                 bitonic_sort_segmented_keys
 * Returns as bitonic_sort_segmented_keys; BITONIC_EINVAL also for values
 * NULL with nseg > 0.
 */
int bitonic_sort_segmented_pairs(void* keys, int32_t* values, const int64_t* offsets,
                                 int64_t nseg, int64_t max_seg_len, int key_type,
                                 int ascending, void* stream);

/*
 * Plans.  A plan fixes how the k(k+1)/2 steps of the network map onto
 * kernel launches; every plan gives the same sorted keys.
 *   BITONIC_PLAN_BASIC      one launch per step, one compare-exchange per
 *                           thread in global memory (section 3.3)
 *   BITONIC_PLAN_SEMI       steps whose stride fits in an LDS tile run in one
 *                           launch per tile phase; longer strides one launch
 *                           per step (section 4.1)
 *   BITONIC_PLAN_OPTIMIZED  register-resident tile sort and merges, and up to
 *                           `fuse` consecutive long-stride steps per HBM pass
 *                           (sections 4.1 and 4.2); passes of nine and ten
 *                           steps split each column of keys over two or four
 *                           lanes of a wave (tuning value "lane_pass")
 */
enum bitonic_plan_kind {
  BITONIC_PLAN_AUTO = 0,
  BITONIC_PLAN_BASIC = 1,
  BITONIC_PLAN_SEMI = 2,
  BITONIC_PLAN_OPTIMIZED = 3
};

typedef struct bitonic_plan {
  int kind;                /* enum bitonic_plan_kind */
  int tile_log2;           /* keys per on-chip tile = 2^tile_log2, 11..15 for
                              the optimized plan, 1..13 for semi (0 = library
                              choice: by n for the optimized plan, see
                              bitonic_plan_tile_log2; 12 for semi) */
  int fuse;                /* max long-stride steps per HBM pass, 1..10
                              (0 = library choice, 10); at most 8 are used
                              for an array off a 16-byte boundary, in
                              phases above 30, or with lane passes off --
                              at most 7 then when n is not a power of two */
  int merge_blocks_per_cu; /* tile-merge workgroups per compute unit, 1..16,
                              each looping over its tiles with the next
                              tile's loads in flight; -1 = one tile per
                              workgroup (0 = library choice, 2) */
} bitonic_plan;

/*
 * The 8-byte sorts with an explicit plan: an 8-byte key_type (I64, U64,
 * F64) sorts keys (bitonic_sort_keys64; values must be NULL), a 4-byte one
 * sorts pairs (bitonic_sort_pairs).  The plan's kind
 * must be BITONIC_PLAN_AUTO or BITONIC_PLAN_OPTIMIZED, its tile_log2 11..13
 * (elements per tile), its fuse 1..8 (7 and 8 split each column over two
 * or four lanes, for n a power of two and phases up to 29; otherwise at
 * most 6 are used); merge_blocks_per_cu is ignored (one tile per
 * workgroup).  Library choices (0): tile_log2 13, fuse 8 (tuning values
 * "wide_tile_log2" and "wide_fuse").
 */
int bitonic_sort_wide_plan(void* keys, int32_t* values, int64_t n, int key_type, int ascending,
                           const bitonic_plan* plan, void* stream);

/*
 * The tile size (log2 keys) the 4-byte sort of n keys uses under `plan`
 * (NULL = BITONIC_PLAN_AUTO): the plan's or the tuned value if set, else the
 * library's choice by n -- 2^12 keys for n <= 2^16, 2^13 for n <= 2^20, 2^14
 * above (measured on MI355X).  0 for the Basic plan, -1 for a bad plan or n.
 */
int bitonic_plan_tile_log2(int64_t n, const bitonic_plan* plan);

/* Launches of an 8-byte sort of n elements under `plan` (-1: bad plan or n). */
int64_t bitonic_wide_plan_passes(int64_t n, const bitonic_plan* plan);

/*
 * bitonic_sort_i32 with an explicit plan (used for the section 5 ablation
 * and by the autotuner).  plan == NULL means BITONIC_PLAN_AUTO.
 * Returns BITONIC_EINVAL for a plan the library does not implement.
 */
int bitonic_sort_plan_i32(int32_t* keys, int64_t n, int ascending,
                          const bitonic_plan* plan, void* stream);

/*
 * Run only phases 1..last_phase of the network (flip arrangement) on
 * keys[0, n): afterwards every aligned block of 2^last_phase keys (the last
 * one cut at n) is sorted, the state section 3.1 describes after that phase.
 * last_phase >= log2(N) sorts fully.  For tests of intermediate states.
 */
int bitonic_network_phases_i32(int32_t* keys, int64_t n, int ascending,
                               int last_phase, const bitonic_plan* plan,
                               void* stream);

/*
 * Number of passes the plan makes over the keys for n keys (each pass reads
 * and writes every key once); -1 on a bad argument.  For n >= 2 the
 * optimized plan makes 1 + sum over phases p > t of (ceil((p - t) / f) + 1)
 * passes.  A long-stride pass over a non-power-of-two n may run as two
 * kernels: one over the 2^(q+f)-key blocks wholly below n, one over the
 * block that straddles n.
 */
int64_t bitonic_plan_passes(int64_t n, const bitonic_plan* plan);

/*
 * Launch description, for measurement.  For each launch i of the plan for n
 * keys (i < cap) writes kinds[i] (enum bitonic_launch_kind) and fuse[i] (the
 * number of network steps a global pass fuses, 1 for a step launch, else
 * 0); either array may be NULL.  Returns the number of launches, -1 on a bad
 * argument.
 */
enum bitonic_launch_kind {
  BITONIC_LAUNCH_TILE_SORT = 1,   /* phases 1..t on every tile (one HBM pass) */
  BITONIC_LAUNCH_GLOBAL_PASS = 2, /* fused long-stride steps (one HBM pass) */
  BITONIC_LAUNCH_TILE_MERGE = 3,  /* strides 2^(t-1)..1 on every tile (one HBM pass) */
  BITONIC_LAUNCH_LDS_NETWORK = 4, /* LDS network on tiles (one HBM pass) */
  BITONIC_LAUNCH_STEP = 5,        /* one step in global memory (one HBM pass) */
  BITONIC_LAUNCH_SEG_PREP = 6,    /* segmented sort: classify the segments */
  BITONIC_LAUNCH_SEG_SMALL = 7    /* segmented sort: all segments of <= 2^13 keys */
};

int64_t bitonic_plan_describe(int64_t n, const bitonic_plan* plan, int32_t* kinds,
                              int32_t* fuse, int64_t cap);

/*
 * Launch shapes, for checks of the planners; nothing is enqueued and no
 * device is touched.  For launch i (i < cap) of a sort of n elements laid out
 * as `layout`, under `plan` (NULL = the library's choice; ignored by the
 * segmented layouts, which follow the tuning values), writes shapes[i]:
 *   kind         enum bitonic_launch_kind
 *   fuse         network steps of a global pass, 1 for a step, else 0
 *   q            lowest index bit a global pass or step works on (its steps
 *                cover bits q + fuse - 1 .. q, segment-local for segmented
 *                sorts); log2 of the tile for tile, LDS and small-segment
 *                launches
 *   mirror       1 if the launch's first step is the mirror step of a phase
 *                (a tile merge with mirror 1 performs all of phase q on its
 *                2^q-key tiles: phase t+1 of a sort with 2^t-key tiles)
 *   elem_bytes   bytes per element in each array: 4 (4-byte keys; pairs,
 *                whose keys and values are two 4-byte arrays) or 8 (8-byte keys)
 *   offset_bits  width of the byte offsets the kernel adds to a row or tile
 *                start: 32, or 64 where it indexes through 64-bit pointers
 * A kernel stays in range when every row of 2^q elements spans at most
 * 2^offset_bits bytes.  Layouts: BITONIC_LAYOUT_KEYS32 (4-byte keys,
 * 16-byte aligned), BITONIC_LAYOUT_KEYS32_UNALIGNED (4-byte keys off a
 * 16-byte boundary), BITONIC_LAYOUT_KEYS64, BITONIC_LAYOUT_PAIRS, and the
 * segmented sorts BITONIC_LAYOUT_SEG_KEYS32, BITONIC_LAYOUT_SEG_PAIRS,
 * BITONIC_LAYOUT_SEG_KEYS64, whose longest segment holds n elements (the
 * bound of bitonic_sort_segmented_bounded_i32).  Returns the number of
 * launches, or -1 for a bad argument (n < 0, n > 2^31, a bad plan or layout).
 */
typedef struct bitonic_launch_shape {
  int32_t kind;
  int32_t fuse;
  int32_t q;
  int32_t mirror;
  int32_t elem_bytes;
  int32_t offset_bits;
} bitonic_launch_shape;

enum bitonic_layout {
  BITONIC_LAYOUT_KEYS32 = 0,
  BITONIC_LAYOUT_KEYS32_UNALIGNED = 1,
  BITONIC_LAYOUT_KEYS64 = 2,
  BITONIC_LAYOUT_PAIRS = 3,
  BITONIC_LAYOUT_SEG_KEYS32 = 4,
  BITONIC_LAYOUT_SEG_PAIRS = 5,
  BITONIC_LAYOUT_SEG_KEYS64 = 6
};

int64_t bitonic_plan_shapes(int64_t n, int layout, const bitonic_plan* plan,
                            bitonic_launch_shape* shapes, int64_t cap);

/*
 * bitonic_sort_plan_i32 that also records HIP events on `stream`:
 * events[0] before the first launch and events[i + 1] right after launch i
 * (for i + 1 < nevents).  `events` is an array of hipEvent_t created by the
 * caller.  Used to time every kernel of a sort on the device.
 */
int bitonic_sort_plan_events_i32(int32_t* keys, int64_t n, int ascending,
                                 const bitonic_plan* plan, void** events,
                                 int64_t nevents, void* stream);

/*
 * Enqueue only launches [first, first + count) of the plan for n keys (the
 * order of bitonic_plan_describe).  Running a subset leaves the keys in an
 * intermediate state; it exists to time single kernels on the device.  In
 * the optimized plan the first kernel maps the keys into the sorting domain
 * and the last maps them back (the identity for ascending int32), so an
 * intermediate state holds mapped keys.
 */
int bitonic_sort_plan_launches_i32(int32_t* keys, int64_t n, int ascending,
                                   const bitonic_plan* plan, int64_t first,
                                   int64_t count, void* stream);

/*
 * Tuning.  bitonic_set_tuning(tile_log2, fuse, merge_blocks_per_cu) changes
 * the library's default plan for BITONIC_PLAN_AUTO (values as in
 * bitonic_plan; 0 keeps the current value).  bitonic_set_tuning_value sets
 * one value by name: "tile_log2" (0 restores the choice by n), "fuse",
 * "merge_blocks_per_cu" (as in bitonic_plan), "seg_blocks_per_cu" (1..16, workgroups per compute unit of
 * the persistent small-segment kernel), "seg_pass_blocks_per_cu" (1..32,
 * workgroups per compute unit of the big-segment passes, default 8),
 * "seg_fuse" (1..5, steps per big-segment pass, default 5), "validate" (0 or 1:
 * offsets validation, see bitonic_validation_error), "tile_lane_steps"
 * (1, the default: the tile sort runs its phases up to 9 as cross-lane
 * compare-exchanges inside each wave; 0: every phase through LDS regroups),
 * "phase_merge" (1, the default: phase t+1 after the tile sort of 2^t-element
 * tiles runs as one launch on 2^(t+1)-element tiles -- for single arrays of
 * 4-byte keys on a 16-byte boundary with t <= 14, for the 8-byte sorts, and
 * for the big segments of every segmented sort; 0: a one-step pass and a
 * tile merge), "phase_blocks_per_cu" (-1..16:
 * tile-phase workgroups per compute unit, each looping over its tiles,
 * default 1; -1 one tile per workgroup; 0 as the tile merges),
 * "lane_pass" (7, the default: passes of eight and nine steps hold 2^7 keys
 * of a column per lane over two and four lanes, ten steps 2^8 over four;
 * 8: only nine and ten steps as lane passes, 2^8 keys per lane; 9: eight
 * steps as with 7, nine and ten with each column over the four waves of a
 * workgroup, exchanging through LDS (longer memory runs: faster once the
 * keys no longer fit the Infinity Cache); 0: no lane passes, so at most
 * eight steps per pass),
 * "sort_tile_log2" (0, the default, or 11..15: when larger than the
 * optimized plan's tile 2^t, the tile sort takes 2^s-key tiles, phases
 * 1..s in one launch, and every later phase passes down to stride 2^t and
 * merges 2^t-key tiles -- one launch fewer than tiles of 2^t with the tile
 * phase, for a longer tile sort; for n a power of two on a 16-byte
 * boundary, with explicit optimized plans too),
 * "wide_tile_log2" (11..13) or
 * "wide_fuse" (1..8) (the 8-byte sorts' plan); bitonic_get_tuning_value
 * reads one.
 * Size buckets: "tile_log2@k", "fuse@k", "merge_blocks_per_cu@k",
 * "lane_pass@k" and "sort_tile_log2@k" (k = ceil(log2 n), 0..31) set the
 * 4-byte sort's plan for that size only (0 removes the entry); a bucket's
 * entries take precedence over the global values, an explicit plan's tile,
 * fuse and merge grid over both.
 * bitonic_load_tuning reads "<name> <value>" lines (the autotuner's output
 * file; '#' starts a comment).  A line "cus <count>" ties the file to
 * devices with that many compute units: on the current device with another
 * count nothing is applied and BITONIC_EUNSUPPORTED is returned.  The file
 * named by the environment variable BITONIC_TUNE_FILE, if set, is loaded
 * once before the first sort.  All return BITONIC_OK or BITONIC_EINVAL; they
 * are not thread-safe with concurrent sorts.
 */
int bitonic_set_tuning(int tile_log2, int fuse, int merge_blocks_per_cu);
int bitonic_set_tuning_value(const char* key, int value);
int bitonic_get_tuning_value(const char* key, int* value);
int bitonic_load_tuning(const char* path);

/*
 * HIP graphs.  A bitonic_graph is a captured launch sequence, replayed with
 * one call and no per-kernel host work.  The device pointers (and n, nseg,
 * the bound, the direction and the plan) are fixed at capture; the keys and
 * offsets they point to may change between replays (an offsets table of
 * fixed capacity can describe fewer segments by making the rest empty).
 *
 * bitonic_graph_capture_sort_i32: the single-array sort of keys[0, n).
 * bitonic_graph_capture_segmented_i32: the segmented sort with a host bound
 *   max_seg_len >= 1 on the segment length; the graph owns its own scratch
 *   buffer (allocated here), so replays of one graph must not overlap each
 *   other, while different graphs may run concurrently.
 * bitonic_graph_launch enqueues one replay on `stream` (hipStream_t).
 * bitonic_graph_destroy frees the graph (and its scratch) -- only after every
 * replay has finished.
 * Returns BITONIC_OK, BITONIC_EINVAL, BITONIC_ENOMEM, BITONIC_ELAUNCH or
 * BITONIC_EDEVICE (capture failed).
 */
typedef struct bitonic_graph bitonic_graph;
int bitonic_graph_capture_sort_i32(bitonic_graph** out, int32_t* keys, int64_t n,
                                   int ascending, const bitonic_plan* plan);
int bitonic_graph_capture_segmented_i32(bitonic_graph** out, int32_t* keys,
                                        const int64_t* offsets, int64_t nseg,
                                        int64_t max_seg_len, int ascending);
int bitonic_graph_launch(bitonic_graph* g, void* stream);
int bitonic_graph_destroy(bitonic_graph* g);

/*
 * Input generator (not part of the sorting method): writes
 * out[i] = (int32)(splitmix64(seed + (start + i + 1) * 0x9E3779B97F4A7C15) >> 32)
 * for i in [0, n), the counter-based SplitMix64 stream of Steele, Lea and
 * Flood (2014).  Device pointer, asynchronous on `stream`.
 */
int bitonic_keygen_i32(int32_t* out, int64_t n, uint64_t seed, int64_t start,
                       void* stream);

/* Library version string and the gfx target it was built for. */
const char* bitonic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BITONIC_MI355X_H */
