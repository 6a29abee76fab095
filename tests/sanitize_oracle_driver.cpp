// Host sanitizer run of the CPU oracle (test infrastructure): every entry
// point on small and edge-case inputs, built with AddressSanitizer and
// UndefinedBehaviorSanitizer.  The results are checked only for being sorted
// here; the pins in test_oracle*.py fix the values.  Prints "ok" on success.
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
typedef void (*oracle_stage_hook)(void* ctx, int phase, int step, const int32_t* keys,
                                  int64_t len);
int oracle_sort_i32(int32_t* keys, int64_t n, int ascending);
int oracle_sort_i32_parallel(int32_t* keys, int64_t n, int ascending, int threads);
int oracle_sort_u32(uint32_t* keys, int64_t n, int ascending);
int oracle_sort_f32_bits(uint32_t* keys, int64_t n, int ascending);
int oracle_sort_segmented_keys(uint32_t* keys, const int64_t* offsets, int64_t nseg, int key_type,
                               int ascending);
int oracle_sort_keys64(uint64_t* keys, int64_t n, int key_type, int ascending);
int oracle_sort_pairs(uint32_t* keys, int32_t* values, int64_t n, int key_type, int ascending);
int oracle_sort_segmented_i32(int32_t* keys, const int64_t* offsets, int64_t nseg, int ascending);
int oracle_bitonic_i32(int32_t* keys, int64_t n, int ascending, int variant,
                       oracle_stage_hook hook, void* ctx, int64_t* steps_out, int64_t* cmp_out);
int64_t oracle_step_pairs(int64_t N, int variant, int phase, int step, int64_t* lo, int64_t* hi,
                          int8_t* up, int64_t cap);
int oracle_bitonic_merge_i32(int32_t* keys, int64_t len);
int oracle_bitonic_segmented_i32(int32_t* keys, const int64_t* offsets, int64_t nseg,
                                 int ascending);
int oracle_bitonic_batch_i32(int32_t* keys, int64_t n, int64_t count, int ascending, int variant);
}

static uint64_t rng = 0x9E3779B97F4A7C15ull;
static uint32_t next32() {
  rng ^= rng << 13;
  rng ^= rng >> 7;
  rng ^= rng << 17;
  return (uint32_t)(rng >> 16);
}

static int fails = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed: %s line %d\n", #c, __LINE__); \
      ++fails;                                                    \
    }                                                             \
  } while (0)

static void hook(void* ctx, int, int, const int32_t*, int64_t) { ++*static_cast<int*>(ctx); }

int main() {
  const int64_t sizes[] = {0, 1, 2, 3, 5, 7, 8, 9, 31, 33, 100, 255, 256, 257, 1000, 4097};
  for (int64_t n : sizes) {
    std::vector<int32_t> a(n);
    for (auto& v : a) v = (int32_t)next32();
    for (int asc = 0; asc < 2; ++asc) {
      std::vector<int32_t> s = a;
      CHECK(oracle_sort_i32(s.data(), n, asc) == 0);
      CHECK(asc ? std::is_sorted(s.begin(), s.end()) : std::is_sorted(s.rbegin(), s.rend()));
      for (int th : {1, 3, 16}) {
        std::vector<int32_t> p = a;
        CHECK(oracle_sort_i32_parallel(p.data(), n, asc, th) == 0);
        CHECK(p == s);
      }
      for (int variant = 0; variant < 3; ++variant) {
        std::vector<int32_t> b = a;
        int seen = 0;
        int64_t steps = 0, cmps = 0;
        CHECK(oracle_bitonic_i32(b.data(), n, asc, variant, hook, &seen, &steps, &cmps) == 0);
        CHECK(b == s);
      }
      std::vector<uint32_t> u(n);
      for (int64_t i = 0; i < n; ++i) u[i] = (uint32_t)a[i];
      CHECK(oracle_sort_u32(u.data(), n, asc) == 0);
      CHECK(oracle_sort_f32_bits(u.data(), n, asc) == 0);
      std::vector<uint64_t> w(n);
      for (int64_t i = 0; i < n; ++i) w[i] = ((uint64_t)next32() << 32) | next32();
      for (int kt = 3; kt <= 5; ++kt) CHECK(oracle_sort_keys64(w.data(), n, kt, asc) == 0);
      std::vector<int32_t> vals(n);
      for (int64_t i = 0; i < n; ++i) vals[i] = (int32_t)i;
      for (int kt = 0; kt <= 2; ++kt) CHECK(oracle_sort_pairs(u.data(), vals.data(), n, kt, asc) == 0);
    }
  }
  // segmented: empty, single and uneven segments at an offset
  {
    const int64_t off[] = {3, 3, 4, 9, 9, 300, 1030};
    const int64_t nseg = 6;
    std::vector<int32_t> a(1040);
    for (auto& v : a) v = (int32_t)next32();
    std::vector<int32_t> b = a, c = a;
    CHECK(oracle_sort_segmented_i32(b.data(), off, nseg, 1) == 0);
    CHECK(oracle_bitonic_segmented_i32(c.data(), off, nseg, 1) == 0);
    CHECK(b == c);
    std::vector<uint32_t> u(a.begin(), a.end());
    for (int kt = 0; kt <= 2; ++kt) CHECK(oracle_sort_segmented_keys(u.data(), off, nseg, kt, 0) == 0);
  }
  // step pairs, merge, batch
  for (int64_t N : {2, 8, 64, 1024}) {
    int k = 0;
    while ((int64_t(1) << k) < N) ++k;
    std::vector<int64_t> lo(N), hi(N);
    std::vector<int8_t> up(N);
    for (int p = 1; p <= k; ++p)
      for (int st = 1; st <= p; ++st)
        for (int variant = 0; variant < 2; ++variant)
          CHECK(oracle_step_pairs(N, variant, p, st, lo.data(), hi.data(), up.data(), N) == N / 2);
    std::vector<int32_t> m(N);
    for (int64_t i = 0; i < N; ++i) m[i] = (int32_t)(i < N / 2 ? i : N - i);
    CHECK(oracle_bitonic_merge_i32(m.data(), N) == 0);
    CHECK(std::is_sorted(m.begin(), m.end()));
  }
  {
    std::vector<int32_t> batch(7 * 128);
    for (auto& v : batch) v = (int32_t)(next32() & 1);
    CHECK(oracle_bitonic_batch_i32(batch.data(), 7, 128, 1, 2) == 0);
  }
  // argument errors
  CHECK(oracle_sort_i32(nullptr, 5, 1) != 0);
  CHECK(oracle_sort_i32_parallel(nullptr, 5, 1, 2) != 0);
  CHECK(oracle_bitonic_i32(nullptr, 3, 1, 0, nullptr, nullptr, nullptr, nullptr) != 0);
  CHECK(oracle_step_pairs(1, 0, 1, 1, nullptr, nullptr, nullptr, 0) < 0);
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
