// Segmented-sort kernels instantiated for one storage type (seg_kernels.hpp).
#include "seg_kernels.hpp"

namespace bitonic {

void seg_run_pairs(const SegData& d, const SegLaunch& l, const int64_t* offsets, const SegScratch& sc,
                   hipStream_t st) {
  seg_run(Pairs{d.keys, d.values}, d.cd64, l, offsets, sc, st);
}

}  // namespace bitonic
