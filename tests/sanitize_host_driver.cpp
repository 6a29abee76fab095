// Host sanitizer run of the library's host code (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only): the planners through
// every host-only entry point of include/bitonic.h (launch counts, launch
// shapes, tuning values and files, argument checks that return before any
// device work), the scratch-cache policy with a counting allocator, and the
// CPU emulator of the tile programs.  No GPU is touched.  Prints "ok".
#include <stdint.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bitonic.h"
#include "../paper_1506_01446_amd/csrc/scratch_cache.hpp"

extern "C" {
int emulate_tile(int L, int r, int kind, int32_t* tile, uint32_t valid);
int worst_bank_conflict_lanes(int L, int r, int kind, int banks, int lanes);
int in_wave_regroups(int L, int r, int kind, int* exact);
}

static int fails = 0;
#define CHECK(c)                                                        \
  do {                                                                  \
    if (!(c)) {                                                         \
      std::fprintf(stderr, "check failed: %s line %d\n", #c, __LINE__); \
      ++fails;                                                          \
    }                                                                   \
  } while (0)

struct CountingAlloc {
  std::vector<void*>* blocks;
  void* alloc(size_t bytes) {
    void* p = std::malloc(bytes);
    if (p) blocks->push_back(p);
    return p;
  }
};

int main() {
  // planners: counts, descriptions and shapes over sizes and plans
  const int64_t sizes[] = {0, 1, 2, 3, 1000, 4097, (1 << 16) + 5, 1 << 20, 10000000,
                           (int64_t(1) << 30) + (1 << 20), int64_t(1) << 31};
  std::vector<bitonic_launch_shape> shapes(4096);
  std::vector<int32_t> kinds(4096), fuse(4096);
  for (int64_t n : sizes) {
    for (int kind = 0; kind <= 3; ++kind)
      for (int t : {0, 11, 13, 15})
        for (int f : {0, 1, 5, 8, 9, 10}) {
          bitonic_plan plan{kind, kind == 2 && t > 13 ? 12 : t, f, 0};
          const int64_t m = bitonic_plan_passes(n, &plan);
          if (m < 0) continue;
          CHECK(bitonic_plan_describe(n, &plan, kinds.data(), fuse.data(), 4096) == m);
          CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS32, &plan, shapes.data(), 4096) == m);
          CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS32_UNALIGNED, &plan, shapes.data(), 4096) >= 0);
          CHECK(bitonic_plan_tile_log2(n, &plan) >= 0);
        }
    for (int t : {11, 12, 13})
      for (int f : {1, 6}) {
        bitonic_plan plan{BITONIC_PLAN_OPTIMIZED, t, f, 0};
        const int64_t m = bitonic_wide_plan_passes(n, &plan);
        CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS64, &plan, shapes.data(), 4096) == m);
        CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_PAIRS, &plan, shapes.data(), 4096) == m);
      }
    for (int lay = BITONIC_LAYOUT_SEG_KEYS32; lay <= BITONIC_LAYOUT_SEG_KEYS64; ++lay)
      CHECK(bitonic_plan_shapes(n, lay, nullptr, shapes.data(), 4096) >= 0);
  }
  // lane-pass modes
  for (int mode : {0, 7, 8}) {
    CHECK(bitonic_set_tuning_value("lane_pass", mode) == BITONIC_OK);
    bitonic_plan plan{BITONIC_PLAN_OPTIMIZED, 11, 10, 0};
    for (int64_t n : sizes)
      CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS32, &plan, shapes.data(), 4096) ==
            bitonic_plan_passes(n, &plan));
  }
  CHECK(bitonic_set_tuning_value("lane_pass", 5) == BITONIC_EINVAL);
  for (int on : {0, 1}) {
    CHECK(bitonic_set_tuning_value("phase_merge", on) == BITONIC_OK);
    bitonic_plan plan{BITONIC_PLAN_OPTIMIZED, 14, 8, 0};
    for (int64_t n : sizes)
      CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS32, &plan, shapes.data(), 4096) ==
            bitonic_plan_passes(n, &plan));
  }
  // tile-sort tiles larger than the merge tile
  for (int s : {0, 13, 15}) {
    CHECK(bitonic_set_tuning_value("sort_tile_log2", s) == BITONIC_OK);
    bitonic_plan plan{BITONIC_PLAN_OPTIMIZED, 12, 10, 0};
    for (int64_t n : sizes)
      CHECK(bitonic_plan_shapes(n, BITONIC_LAYOUT_KEYS32, &plan, shapes.data(), 4096) ==
            bitonic_plan_passes(n, &plan));
  }
  CHECK(bitonic_set_tuning_value("sort_tile_log2", 16) == BITONIC_EINVAL);
  CHECK(bitonic_set_tuning_value("sort_tile_log2", 0) == BITONIC_OK);
  CHECK(bitonic_set_tuning_value("lane_pass", 7) == BITONIC_OK);
  CHECK(bitonic_plan_shapes(-1, 0, nullptr, nullptr, 0) == -1);
  CHECK(bitonic_plan_shapes(5, 99, nullptr, nullptr, 0) == -1);
  // shapes into a too-small array: the count still comes back, nothing overflows
  CHECK(bitonic_plan_shapes(1 << 24, BITONIC_LAYOUT_KEYS32, nullptr, shapes.data(), 3) == 20);

  // argument checks that return before any device work
  CHECK(bitonic_sort_i32(nullptr, -1, 1, nullptr) == BITONIC_EINVAL);
  CHECK(bitonic_sort_keys64(nullptr, 5, BITONIC_KEY_I64, 1, nullptr) == BITONIC_EINVAL);
  CHECK(bitonic_sort_pairs(nullptr, nullptr, 2, BITONIC_KEY_I32, 1, nullptr) == BITONIC_EINVAL);
  CHECK(bitonic_sort_segmented_i32(nullptr, nullptr, -1, 1, nullptr) == BITONIC_EINVAL);
  CHECK(bitonic_sort_segmented_noalloc_i32(nullptr, nullptr, int64_t(1) << 18, 8, 1, nullptr) ==
        BITONIC_EUNSUPPORTED);
  CHECK(bitonic_segmented_default_bound(nullptr, 4) == -1);
  CHECK(std::strlen(bitonic_status_string(12345)) > 0);

  // tuning values and a tuning file with comments, buckets and a bad line
  int v = 0;
  CHECK(bitonic_set_tuning_value("fuse@24", 6) == BITONIC_OK);
  CHECK(bitonic_get_tuning_value("fuse@24", &v) == BITONIC_OK && v == 6);
  CHECK(bitonic_set_tuning_value("fuse@99", 6) == BITONIC_EINVAL);
  CHECK(bitonic_set_tuning_value("@", 6) == BITONIC_EINVAL);
  CHECK(bitonic_set_tuning_value("tile_log2@", 6) == BITONIC_EINVAL);
  CHECK(bitonic_set_tuning_value("fuse@24", 0) == BITONIC_OK);
  {
    char path[] = "/tmp/bitonic_san_tuneXXXXXX";
    const int fd = mkstemp(path);
    CHECK(fd >= 0);
    FILE* f = fdopen(fd, "w");
    std::fprintf(f, "# comment\nseg_fuse 4 # trailing\n\ntile_log2@20 13\n");
    std::fprintf(f, "a_key_that_is_much_longer_than_the_sixty_three_characters_the_loader_reads_at_once 1\n");
    std::fprintf(f, "fuse 3 extra\n");
    std::fclose(f);
    CHECK(bitonic_load_tuning(path) == BITONIC_EINVAL);
    CHECK(bitonic_get_tuning_value("seg_fuse", &v) == BITONIC_OK && v == 4);
    CHECK(bitonic_get_tuning_value("tile_log2@20", &v) == BITONIC_OK && v == 13);
    std::remove(path);
    bitonic_set_tuning_value("tile_log2@20", 0);
    bitonic_set_tuning_value("seg_fuse", 5);
  }

  // the scratch-cache policy: growth retires, never frees
  {
    std::vector<void*> blocks;
    bitonic::ScratchCache<CountingAlloc> cache(CountingAlloc{&blocks});
    int s1 = 0, s2 = 0;
    void* a = cache.get(0, &s1, 100);
    CHECK(a != nullptr && cache.get(0, &s1, 1000) == a);
    void* b = cache.get(0, &s1, (size_t(1) << 21));
    CHECK(b != a && cache.retired_count() == 1);
    CHECK(cache.get(0, &s2, 10) != b);
    CHECK(cache.get(1, &s1, 10) != b);
    CHECK(blocks.size() == 4);
    for (void* p : blocks) std::free(p);
  }

  // the CPU emulator on every program the kernels instantiate
  for (int kind : {0, 1, 2, 3, 4, 6})
    for (int L = (kind == 2 || kind == 6 ? 5 : 11); L <= (kind == 2 || kind == 3 || kind == 6 ? 13 : 15); ++L) {
      std::vector<int32_t> tile(size_t(1) << L);
      for (size_t i = 0; i < tile.size(); ++i) tile[i] = (int32_t)((i * 2654435761u) >> 7);
      CHECK(emulate_tile(L, 5, kind, tile.data(), (uint32_t)tile.size() - 3) >= 0);
      int exact = 0;
      CHECK(in_wave_regroups(L, 5, kind, &exact) >= 0);
      if (L > 5) CHECK(worst_bank_conflict_lanes(L, 5, kind, 32, 32) >= 1);
    }
  for (int L = 11; L <= 13; ++L)
    for (int kind : {2, 3}) {
      std::vector<int32_t> tile(size_t(1) << L, 7);
      CHECK(emulate_tile(L, 4, kind, tile.data(), 100) >= 0);
    }

  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}
