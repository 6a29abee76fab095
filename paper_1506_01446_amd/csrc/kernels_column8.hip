// Eight-step one-column passes of the 4-byte sort, without the mirror step
// (see kernels_column.hip).
#include "column_pass.hpp"
#include "launch.hpp"

namespace bitonic {

void launch_column_pass8_plain(int32_t* keys, uint32_t n, int q, hipStream_t st) {
  launch_column_pass_FM<8, false>(Keys32{keys}, n, q, st);
}

void launch_column_pass8_mirror(int32_t* keys, uint32_t n, int q, hipStream_t st);

void launch_column_pass8(bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  if (mirror)
    launch_column_pass8_mirror(keys, n, q, st);
  else
    launch_column_pass8_plain(keys, n, q, st);
}

}  // namespace bitonic
