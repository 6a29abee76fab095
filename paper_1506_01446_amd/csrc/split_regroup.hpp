// Tile programs on 8-byte elements with half the LDS: each regroup moves the
// elements' high words through an LDS array of 4-byte words, then their low
// words.  It costs two more synchronisations per regroup than regroup
// (device.hpp) and lets twice as many workgroups share a CU, which for the 2^12..2^13
// element tiles of the 8-byte sorts is the difference between two and four
// workgroups (8 and 16 or 32 waves).
#pragma once

#include "device.hpp"

namespace bitonic {

// regroup of 8-byte elements through an LDS array of PR::LDSW 4-byte words.
template <class PR, int GA, int GB>
__device__ __forceinline__ void regroup_split(int64_t (&x)[PR::R], uint32_t* lds, uint32_t tid) {
  if constexpr (PR::LEAN) asm volatile("" : "+v"(tid));
  const LdsBase<PR, GA> a(tid);
  const LdsBase<PR, GB> b(tid);
  uint32_t hi[PR::R];
  regroup_enter<GA>();
  static_for<0, PR::R>([&](auto J) { lds[a.template at<J>()] = (uint32_t)((uint64_t)x[J] >> 32); });
  regroup_sync<PR, GA, GB>();
  static_for<0, PR::R>([&](auto J) { hi[J] = lds[b.template at<J>()]; });
  // the low words overwrite positions other lanes (other waves, unless the
  // regroup stays inside its wave) read the high words from
  regroup_sync<PR, GA, GB>();
  static_for<0, PR::R>([&](auto J) { lds[a.template at<J>()] = (uint32_t)(uint64_t)x[J]; });
  regroup_sync<PR, GA, GB>();
  static_for<0, PR::R>([&](auto J) {
    x[J] = (int64_t)(((uint64_t)hi[J] << 32) | lds[b.template at<J>()]);
  });
}

template <class PR, int G>
__device__ __forceinline__ void run_from_split(int64_t (&x)[PR::R], uint32_t* lds, uint32_t tid) {
  group_steps<PR, G>(x);
  if constexpr (G + 1 < PR::value.ngroups) {
    regroup_split<PR, G, G + 1>(x, lds, tid);
    run_from_split<PR, G + 1>(x, lds, tid);
  }
}

}  // namespace bitonic
