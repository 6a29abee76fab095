// One-column fused passes of the single-array sort of 4-byte keys: for six to
// eight steps per pass (2^f keys per thread: 64, 128 or 256), and for any
// number of steps when the array does not start on a 16-byte boundary (the
// one-column kernel needs only 4-byte alignment).  Each large
// instantiation has a file of its own so that they compile in parallel:
// f = 6, 7 here, f = 8 in kernels_column8m.hip (with the mirror step) and
// kernels_column8.hip (without).
#include "column_pass.hpp"
#include "launch.hpp"

namespace bitonic {

void launch_column_pass8(bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st);

void launch_column_pass_i32(int f, bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  switch (f) {
    case 1: launch_column_pass_F<1>(mirror, Keys32{keys}, n, q, st); break;
    case 2: launch_column_pass_F<2>(mirror, Keys32{keys}, n, q, st); break;
    case 3: launch_column_pass_F<3>(mirror, Keys32{keys}, n, q, st); break;
    case 4: launch_column_pass_F<4>(mirror, Keys32{keys}, n, q, st); break;
    case 5: launch_column_pass_F<5>(mirror, Keys32{keys}, n, q, st); break;
    case 6: launch_column_pass_F<6>(mirror, Keys32{keys}, n, q, st); break;
    case 7: launch_column_pass_F<7>(mirror, Keys32{keys}, n, q, st); break;
    case 8: launch_column_pass8(mirror, keys, n, q, st); break;
    default: break;
  }
}

}  // namespace bitonic
