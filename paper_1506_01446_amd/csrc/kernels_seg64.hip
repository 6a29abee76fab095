// Segmented-sort kernels instantiated for one storage type (seg_kernels.hpp).
#include "seg_kernels.hpp"

namespace bitonic {

void seg_run_keys64(const SegData& d, const SegLaunch& l, const int64_t* offsets, const SegScratch& sc,
                    hipStream_t st) {
  seg_run(Keys64{d.keys64}, d.cd64, l, offsets, sc, st);
}

}  // namespace bitonic
