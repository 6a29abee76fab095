// Lane passes with 2^8 keys per lane: nine steps (one lane bit) and ten
// (two lane bits); see column_lanes_pass_kernel.
#include "column_pass.hpp"
#include "launch.hpp"

namespace bitonic {

bool launch_column_lanes_pass8(int f, bool waves, bool mirror, int32_t* keys, uint32_t n, int q,
                               hipStream_t st) {
  if (waves) {  // four waves per column (f = 10)
    if (f != 10) return false;
    launch_column_waves_F<8>(mirror, keys, n, q, st);
    return true;
  }
  switch (f) {
    case 9: launch_column_lanes_FG<8, 1>(mirror, keys, n, q, st); return true;
    case 10: launch_column_lanes_FG<8, 2>(mirror, keys, n, q, st); return true;
    default: return false;
  }
}

}  // namespace bitonic
