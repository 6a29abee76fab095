// Lane passes with 2^7 keys per lane: eight steps (one lane bit) and nine
// (two lane bits); see column_lanes_pass_kernel.
#include "column_pass.hpp"
#include "launch.hpp"

namespace bitonic {

bool launch_column_lanes_pass8(int f, bool waves, bool mirror, int32_t* keys, uint32_t n, int q,
                               hipStream_t st);

bool launch_column_lanes_pass(int f, int fr, bool mirror, int32_t* keys, uint32_t n, int q,
                              hipStream_t st) {
  if (!lane_pass_fits(n, q, f)) return false;
  if (fr < 0 && !wave_pass_fits(n, q, f)) return false;
  if (fr == 8 || fr == -8) return launch_column_lanes_pass8(f, fr < 0, mirror, keys, n, q, st);
  if (fr == -7) {  // four waves per column (f = 9)
    if (f != 9) return false;
    launch_column_waves_F<7>(mirror, keys, n, q, st);
    return true;
  }
  if (fr != 7) return false;
  switch (f) {
    case 8: launch_column_lanes_FG<7, 1>(mirror, keys, n, q, st); return true;
    case 9: launch_column_lanes_FG<7, 2>(mirror, keys, n, q, st); return true;
    default: return false;
  }
}

}  // namespace bitonic
