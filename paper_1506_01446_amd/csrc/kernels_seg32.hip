// Segmented-sort kernels instantiated for one storage type (seg_kernels.hpp).
#include "seg_kernels.hpp"

namespace bitonic {

void seg_run_keys32(const SegData& d, const SegLaunch& l, const int64_t* offsets, const SegScratch& sc,
                    hipStream_t st) {
  seg_run(Keys32{d.keys}, d.cd, l, offsets, sc, st);
}

}  // namespace bitonic
