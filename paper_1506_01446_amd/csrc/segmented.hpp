// Host-side launcher of the segmented sort (internal interface).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bitonic {

// Enqueue the counter reset and the persistent segmented kernel with `grid`
// workgroups.  `counter` is a device word of the library's scratch.
void launch_segmented(int32_t* keys, const int64_t* offsets, int64_t nseg, int32_t flip,
                      uint32_t* counter, int grid, hipStream_t st);

}  // namespace bitonic
