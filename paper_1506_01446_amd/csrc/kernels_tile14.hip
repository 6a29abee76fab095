// Tile sort and merge kernels of 2^14-key tiles (see tile_kernels.hpp).
#include "tile_kernels.hpp"

namespace bitonic {

void launch_tile_14(int kind, int32_t* keys, uint32_t n, Codec cd, int cx, uint32_t max_blocks,
                    hipStream_t st) {
  launch_tile_L<14>(kind, keys, n, cd, cx, max_blocks, st);
}

}  // namespace bitonic
