// CPU oracle for the bitonic sort of 32-bit integer keys.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file: only the test suite, the smoke check and the benchmark's
// CPU-baseline leg use it.  It shares no code with the HIP library.
//
// Two oracles, both plain and slow on purpose:
//
//  1. oracle_sort_i32 / oracle_sort_segmented_i32 -- the plain definition of
//     what the method computes: the n keys in signed int32 order (std::sort,
//     an introsort, i.e. a quicksort variant, which stands in for the CPU
//     QuickSort baseline of section 5).  Descending is the ascending result
//     read backwards.  A keys-only sort has exactly one correct output.
//
//  2. oracle_bitonic_i32 -- the bitonic sorting network of section 3.1 run
//     scalar, one compare-exchange at a time, in the paper's order: k phases
//     for n = 2^k; phase r sorts the 2^(k-r) subsequences of length 2^r by a
//     bitonic merge of r steps (strides 2^(r-1) ... 1), each step being n/2
//     compare-exchanges (section 3.1, section 3.3).  Counters report the
//     number of steps ("rounds") and of compare-exchanges, whose closed forms
//     are given in section 3.2.
//
//     Variants (all give the same final output):
//       ORACLE_STANDARD      Batcher's network as section 3.1 describes it:
//                            subsequences alternate direction within a phase
//                            (block containing i ascending iff bit r of i is
//                            0), every step compares i with i XOR stride.
//                            Non-power-of-two n is padded with INT32_MAX
//                            sentinels, materialised.
//       ORACLE_FLIP          Same comparators in the "flip" arrangement: the
//                            first step of phase r compares i with its mirror
//                            i XOR (2^r - 1) inside the 2^r block, and every
//                            comparator puts the smaller key at the lower
//                            index.  After phase r every aligned 2^r block is
//                            ascending.  Sentinels materialised.
//       ORACLE_FLIP_VIRTUAL  ORACLE_FLIP with the sentinels never stored:
//                            every comparator whose upper index is >= n is
//                            skipped, because an absent +infinity partner
//                            would leave the lower key where it is.
//
//     Descending order: ORACLE_STANDARD runs every block in the opposite
//     direction; INT32_MAX sentinels then gather at the front, so the answer
//     is x[N-n .. N).  The flip variants put the larger key at the lower
//     index; the virtual one then treats the absent sentinels as INT32_MIN,
//     which keeps them at the back and the answer at x[0 .. n).
//
//  3. oracle_sort_keys64 / oracle_sort_pairs -- the plain definitions for
//     8-byte keys and for (key, value) pairs (the paper's future work names
//     other key types; the pair order is a definition of this library: by
//     key, then by value).
//
// Readings of the paper taken here:
//  * "alternating descending and ascending" is read with the first block
//    ascending (block ascending iff bit r of the index is 0); either reading
//    gives the same final output.
//  * "[k.1]th phase" is the (k-1)th phase; phase k sorts A.
//  * n that is not a power of two: padded with INT32_MAX up to N = 2^k.
//  * keys are signed 32-bit integers.

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

namespace {

constexpr int32_t kSentinel = INT32_MAX;

// Smallest power of two >= n (1 for n <= 1).
int64_t padded_size(int64_t n) {
  int64_t N = 1;
  while (N < n) N <<= 1;
  return N;
}

int log2_exact(int64_t N) {
  int k = 0;
  while ((int64_t(1) << k) < N) ++k;
  return k;
}

#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

// One compare-exchange: afterwards x[lo_pos] holds the key that belongs at
// the lower position for the requested direction.
inline void compare_exchange(int32_t* x, int64_t i, int64_t j, bool up) {
#if ORACLE_MUTANT == 4
  // planted mistake: keys compared as unsigned integers
  const bool greater = uint32_t(x[i]) > uint32_t(x[j]);
#else
  const bool greater = x[i] > x[j];
#endif
  if (greater == up) std::swap(x[i], x[j]);
}

}  // namespace

extern "C" {

typedef void (*oracle_stage_hook)(void* ctx, int phase, int step,
                                  const int32_t* x, int64_t len);

enum { ORACLE_STANDARD = 0, ORACLE_FLIP = 1, ORACLE_FLIP_VIRTUAL = 2 };

// Plain definition.  Returns 0, or -1 for a bad argument.
int oracle_sort_i32(int32_t* keys, int64_t n, int ascending) {
  if (n < 0 || (n > 0 && keys == nullptr)) return -1;
  std::sort(keys, keys + n);
  if (!ascending) std::reverse(keys, keys + n);
  return 0;
}

// The same sort on `threads` host threads, as a CPU baseline on all cores
// (section 5 compares against one CPU thread; this is context beyond it):
// std::sort of `threads` contiguous chunks in parallel, then pairwise
// std::inplace_merge of neighbouring runs, each level's merges in parallel.
// The result is the ascending (or reversed) order, as oracle_sort_i32.
int oracle_sort_i32_parallel(int32_t* keys, int64_t n, int ascending, int threads) {
  if (n < 0 || (n > 0 && keys == nullptr) || threads < 1) return -1;
  if (threads > 256) threads = 256;
  const int64_t parts = n < threads ? 1 : threads;
  std::vector<int64_t> cut(parts + 1);
  for (int64_t i = 0; i <= parts; ++i) cut[i] = n * i / parts;
  {
    std::vector<std::thread> pool;
    for (int64_t i = 0; i < parts; ++i)
      pool.emplace_back([&, i] { std::sort(keys + cut[i], keys + cut[i + 1]); });
    for (auto& t : pool) t.join();
  }
  for (int64_t width = 1; width < parts; width *= 2) {
    std::vector<std::thread> pool;
    for (int64_t i = 0; i + width < parts; i += 2 * width) {
      const int64_t a = cut[i], m = cut[i + width];
      const int64_t b = cut[std::min<int64_t>(i + 2 * width, parts)];
      pool.emplace_back([=] { std::inplace_merge(keys + a, keys + m, keys + b); });
    }
    for (auto& t : pool) t.join();
  }
  if (!ascending) std::reverse(keys, keys + n);
  return 0;
}

// IEEE 754-2008 totalOrder on binary32 bit patterns: negative values (sign
// bit set) come before positive ones; among positives a larger magnitude
// field is larger; among negatives a larger magnitude field is smaller.  NaNs
// take their place by their bits (-NaN first, +NaN last), and -0 < +0.
static bool f32_total_less(uint32_t a, uint32_t b) {
  const bool na = (a >> 31) != 0, nb = (b >> 31) != 0;
#if ORACLE_MUTANT == 7
  // planted mistake: negatives ordered by increasing magnitude
  if (na != nb) return na;
  return (a & 0x7FFFFFFFu) < (b & 0x7FFFFFFFu);
#else
  if (na != nb) return na;
  const uint32_t ma = a & 0x7FFFFFFFu, mb = b & 0x7FFFFFFFu;
  return na ? (ma > mb) : (ma < mb);
#endif
}

// Plain definitions for the other 32-bit key types (bit patterns in and out).
int oracle_sort_u32(uint32_t* keys, int64_t n, int ascending) {
  if (n < 0 || (n > 0 && keys == nullptr)) return -1;
  std::sort(keys, keys + n);
  if (!ascending) std::reverse(keys, keys + n);
  return 0;
}

int oracle_sort_f32_bits(uint32_t* keys, int64_t n, int ascending) {
  if (n < 0 || (n > 0 && keys == nullptr)) return -1;
  std::sort(keys, keys + n, f32_total_less);
  if (!ascending) std::reverse(keys, keys + n);
  return 0;
}

// Plain definition for key type t (0 int32, 1 uint32, 2 float32 totalOrder)
// on 32-bit patterns, per segment [offsets[s], offsets[s+1]).
int oracle_sort_segmented_keys(uint32_t* keys, const int64_t* offsets, int64_t nseg,
                               int key_type, int ascending) {
  if (nseg < 0 || (nseg > 0 && offsets == nullptr) || key_type < 0 || key_type > 2) return -1;
  for (int64_t s = 0; s < nseg; ++s)
    if (offsets[s + 1] < offsets[s]) return -1;
  for (int64_t s = 0; s < nseg; ++s) {
    uint32_t* k = keys + offsets[s];
    const int64_t len = offsets[s + 1] - offsets[s];
    const int rc = key_type == 0   ? oracle_sort_i32(reinterpret_cast<int32_t*>(k), len, ascending)
                   : key_type == 1 ? oracle_sort_u32(k, len, ascending)
                                   : oracle_sort_f32_bits(k, len, ascending);
    if (rc) return rc;
  }
  return 0;
}

// totalOrder on binary64 bit patterns, the same rule as for binary32.
static bool f64_total_less(uint64_t a, uint64_t b) {
  const bool na = (a >> 63) != 0, nb = (b >> 63) != 0;
  if (na != nb) return na;
  const uint64_t ma = a & 0x7FFFFFFFFFFFFFFFull, mb = b & 0x7FFFFFFFFFFFFFFFull;
#if ORACLE_MUTANT == 10
  // planted mistake: negatives ordered by increasing magnitude
  return ma < mb;
#else
  return na ? (ma > mb) : (ma < mb);
#endif
}

// Plain definition for 8-byte keys (bit patterns in and out): key_type 3
// int64, 4 uint64, 5 float64 in totalOrder.  Descending is the ascending
// result read backwards.
int oracle_sort_keys64(uint64_t* keys, int64_t n, int key_type, int ascending) {
  if (n < 0 || (n > 0 && keys == nullptr) || key_type < 3 || key_type > 5) return -1;
  if (key_type == 3) {
    int64_t* k = reinterpret_cast<int64_t*>(keys);
#if ORACLE_MUTANT == 9
    // planted mistake: only the low 32 bits of each key are compared
    std::stable_sort(k, k + n, [](int64_t a, int64_t b) { return (uint32_t)a < (uint32_t)b; });
#else
    std::sort(k, k + n);
#endif
  } else if (key_type == 4) {
    std::sort(keys, keys + n);
  } else {
    std::sort(keys, keys + n, f64_total_less);
  }
  if (!ascending) std::reverse(keys, keys + n);
  return 0;
}

// Plain definition of the key-value sort: pairs (keys[i], values[i]) in the
// order of their keys (key_type 0 int32, 1 uint32, 2 float32 totalOrder; in
// the requested direction), pairs with equal keys in ascending order of
// their int32 values.  That order is unique: pairs that compare equal are
// identical.  Keys as bit patterns; both arrays rewritten in that order.
int oracle_sort_pairs(uint32_t* keys, int32_t* values, int64_t n, int key_type, int ascending) {
  if (n < 0 || (n > 0 && (keys == nullptr || values == nullptr)) || key_type < 0 ||
      key_type > 2)
    return -1;
  auto key_less = [key_type](uint32_t a, uint32_t b) {
    if (key_type == 0) return (int32_t)a < (int32_t)b;
    if (key_type == 1) return a < b;
    return f32_total_less(a, b);
  };
  std::vector<int64_t> idx(n);
  for (int64_t i = 0; i < n; ++i) idx[i] = i;
  std::sort(idx.begin(), idx.end(), [&](int64_t i, int64_t j) {
    const uint32_t a = keys[i], b = keys[j];
    if (key_less(a, b)) return ascending != 0;
    if (key_less(b, a)) return ascending == 0;
#if ORACLE_MUTANT == 8
    return values[i] > values[j];  // planted mistake: ties by value descending
#else
    return values[i] < values[j];
#endif
  });
  std::vector<uint32_t> k2(n);
  std::vector<int32_t> v2(n);
  for (int64_t i = 0; i < n; ++i) {
    k2[i] = keys[idx[i]];
    v2[i] = values[idx[i]];
  }
  std::copy(k2.begin(), k2.end(), keys);
  std::copy(v2.begin(), v2.end(), values);
  return 0;
}

// Plain definition, per segment [offsets[s], offsets[s+1]).
int oracle_sort_segmented_i32(int32_t* keys, const int64_t* offsets,
                              int64_t nseg, int ascending) {
  if (nseg < 0 || (nseg > 0 && offsets == nullptr)) return -1;
  for (int64_t s = 0; s < nseg; ++s) {
    if (offsets[s + 1] < offsets[s]) return -1;
  }
  for (int64_t s = 0; s < nseg; ++s) {
    int rc = oracle_sort_i32(keys + offsets[s], offsets[s + 1] - offsets[s],
                             ascending);
    if (rc) return rc;
  }
  return 0;
}

// The scalar network.  Sorts keys[0..n) in place.  *steps_out receives the
// number of steps run (k(k+1)/2 for N = 2^k) and *cmp_out the number of
// compare-exchanges evaluated (N/2 per step; skipped virtual comparators are
// not counted).  hook, if not null, sees the whole working array (length N
// for the materialised variants, n for the virtual one) after every step,
// with the phase r in 1..k and the step index 1..r within the phase.
int oracle_bitonic_i32(int32_t* keys, int64_t n, int ascending, int variant,
                       oracle_stage_hook hook, void* ctx, int64_t* steps_out,
                       int64_t* cmp_out) {
  if (n < 0 || (n > 0 && keys == nullptr)) return -1;
  if (variant < ORACLE_STANDARD || variant > ORACLE_FLIP_VIRTUAL) return -1;
  int64_t steps = 0, cmps = 0;
  const int64_t N = padded_size(n);
  const int k = log2_exact(N);
  const bool asc = ascending != 0;
  const bool virt = variant == ORACLE_FLIP_VIRTUAL;

  std::vector<int32_t> x;
  int32_t* a = keys;
  if (!virt) {
    x.assign(N, kSentinel);
#if ORACLE_MUTANT == 6
    // planted mistake: padding with zeros instead of INT32_MAX
    std::fill(x.begin(), x.end(), 0);
#endif
    if (n > 0) std::memcpy(x.data(), keys, sizeof(int32_t) * n);
    a = x.data();
  }
  const int64_t len = virt ? n : N;

  for (int r = 1; r <= k; ++r) {               // phase r: blocks of 2^r keys
    const int64_t block = int64_t(1) << r;
    for (int step = 1; step <= r; ++step) {    // strides 2^(r-1) ... 1
#if ORACLE_MUTANT == 5
      // planted mistake: the last step of every phase is dropped
      if (step == r && r > 1) { ++steps; continue; }
#endif
      const int64_t stride = block >> step;
      for (int64_t i = 0; i < N; ++i) {
        int64_t j;
        bool up;
        if (variant == ORACLE_STANDARD) {
#if ORACLE_MUTANT == 2
          // planted mistake: stride off by one
          j = i ^ (stride > 1 ? stride - 1 : stride);
#else
          j = i ^ stride;
#endif
          if (j <= i) continue;
#if ORACLE_MUTANT == 1
          // planted mistake: no alternation of block directions
          up = asc;
#else
          up = ((i & block) == 0) == asc;
#endif
        } else {
          if (step == 1) {
            if (i & (block >> 1)) continue;    // i in the lower half
#if ORACLE_MUTANT == 3
            // planted mistake: plain half-cleaner partner instead of the
            // mirror, with every comparator still ascending
            j = i ^ (block >> 1);
#else
            j = i ^ (block - 1);                // mirror inside the block
#endif
          } else {
            j = i ^ stride;
            if (j <= i) continue;
          }
          up = asc;
          if (virt && j >= n) continue;         // absent sentinel partner
        }
        compare_exchange(a, i, j, up);
        ++cmps;
      }
      ++steps;
      if (hook) hook(ctx, r, step, a, len);
    }
  }

  if (!virt && n > 0) {
    // Standard descending: the INT32_MAX sentinels lead, keys are the tail.
    // Flip descending with materialised INT32_MAX sentinels: same.
    const int64_t from = asc ? 0 : N - n;
    std::memcpy(keys, a + from, sizeof(int32_t) * n);
  }
  if (steps_out) *steps_out = steps;
  if (cmp_out) *cmp_out = cmps;
  return 0;
}

// The comparators of one step of the standard network for N = 2^k keys, in
// ascending index order of their lower end: writes up to cap pairs (lo, hi)
// and the direction (1 = smaller key to lo) and returns how many there are.
int64_t oracle_step_pairs(int64_t N, int variant, int phase, int step,
                          int64_t* lo, int64_t* hi, int8_t* up, int64_t cap) {
  if (N < 2 || phase < 1 || step < 1 || step > phase) return -1;
  if ((int64_t(1) << phase) > N) return -1;
  const int64_t block = int64_t(1) << phase;
  const int64_t stride = block >> step;
  int64_t m = 0;
  for (int64_t i = 0; i < N; ++i) {
    int64_t j;
    bool u = true;
    if (variant == ORACLE_STANDARD) {
      j = i ^ stride;
      if (j <= i) continue;
      u = (i & block) == 0;
    } else {
      if (step == 1) {
        if (i & (block >> 1)) continue;
        j = i ^ (block - 1);
      } else {
        j = i ^ stride;
        if (j <= i) continue;
      }
    }
    if (m < cap) {
      lo[m] = i;
      hi[m] = j;
      up[m] = u ? 1 : 0;
    }
    ++m;
  }
  return m;
}

// Bitonic merge of section 3.1 on its own: sorts a bitonic sequence of
// length 2^r (in place) by r half-cleaner steps with strides 2^(r-1) ... 1,
// smaller key to the lower index.  Returns -1 unless len is a power of two.
int oracle_bitonic_merge_i32(int32_t* keys, int64_t len) {
  if (len < 1 || (len & (len - 1)) != 0 || keys == nullptr) return -1;
  for (int64_t stride = len >> 1; stride >= 1; stride >>= 1) {
    for (int64_t i = 0; i < len; ++i) {
      const int64_t j = i ^ stride;
      if (j > i) compare_exchange(keys, i, j, true);
    }
  }
  return 0;
}

// Scalar network per segment (flip arrangement, virtual sentinels).
int oracle_bitonic_segmented_i32(int32_t* keys, const int64_t* offsets,
                                 int64_t nseg, int ascending) {
  if (nseg < 0 || (nseg > 0 && offsets == nullptr)) return -1;
  for (int64_t s = 0; s < nseg; ++s) {
    const int64_t len = offsets[s + 1] - offsets[s];
    if (len < 0) return -1;
    int rc = oracle_bitonic_i32(keys + offsets[s], len, ascending,
                                ORACLE_FLIP_VIRTUAL, nullptr, nullptr, nullptr,
                                nullptr);
    if (rc) return rc;
  }
  return 0;
}

// The scalar network on `count` independent arrays of n keys stored one after
// another (used to sweep every 0-1 input of a given length in one call).
int oracle_bitonic_batch_i32(int32_t* keys, int64_t n, int64_t count,
                             int ascending, int variant) {
  if (n < 0 || count < 0 || (n > 0 && count > 0 && keys == nullptr)) return -1;
  for (int64_t c = 0; c < count; ++c) {
    int rc = oracle_bitonic_i32(keys + c * n, n, ascending, variant, nullptr,
                                nullptr, nullptr, nullptr);
    if (rc) return rc;
  }
  return 0;
}

int oracle_mutant_id(void) { return ORACLE_MUTANT; }

}  // extern "C"
