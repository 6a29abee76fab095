// Eight-step one-column passes of the 4-byte sort, with the mirror step
// (see kernels_column.hip).
#include "column_pass.hpp"
#include "launch.hpp"

namespace bitonic {

void launch_column_pass8_mirror(int32_t* keys, uint32_t n, int q, hipStream_t st) {
  launch_column_pass_FM<8, true>(Keys32{keys}, n, q, st);
}

}  // namespace bitonic
