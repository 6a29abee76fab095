// Key codec shared by the host planner and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bitonic {

// Key codec: enc maps a stored 32-bit key to the sorting domain, dec maps it
// back.  enc(x) = g(x) ^ flip with g(x) = x ^ ((x >> 31) & fmask):
//  - int32:   fmask = 0, flip = 0 (ascending) or -1 (descending: ~ reverses
//             signed order);
//  - uint32:  fmask = 0, flip = INT32_MIN (ascending) or INT32_MAX
//             (descending): toggling the sign bit turns unsigned order into
//             signed order;
//  - float32: fmask = INT32_MAX, flip as for int32: g flips the magnitude bits
//             of negative values, which turns IEEE-754 bit patterns into
//             signed integers in totalOrder (-NaN < -inf < ... < -0 < +0 <
//             ... < +inf < +NaN).  g is its own inverse.
struct Codec {
  int32_t flip;
  int32_t fmask;
  __host__ __device__ __forceinline__ int32_t enc(int32_t x) const {
    return x ^ ((x >> 31) & fmask) ^ flip;
  }
  __host__ __device__ __forceinline__ int32_t dec(int32_t y) const {
    const int32_t z = y ^ flip;
    return z ^ ((z >> 31) & fmask);
  }
};

// The same map on 8-byte elements: enc(x) = x ^ ((x >> 63) & fmask) ^ flip.
//  - int64 / uint64 / float64 keys: as for the 4-byte types, on 64 bits;
//  - pairs: a 4-byte key and a 4-byte value form the element
//    key * 2^32 + (uint32)value; the key word takes the 4-byte key codec and
//    the value word has its sign bit toggled, so the elements sort by key (in
//    the requested direction) and then by value ascending as int32.
struct Codec64 {
  int64_t flip;
  int64_t fmask;
  __host__ __device__ __forceinline__ int64_t enc(int64_t x) const {
    return x ^ ((x >> 63) & fmask) ^ flip;
  }
  __host__ __device__ __forceinline__ int64_t dec(int64_t y) const {
    const int64_t z = y ^ flip;
    return z ^ ((z >> 63) & fmask);
  }
};

inline bool codec_is_identity(Codec c) { return c.flip == 0 && c.fmask == 0; }
inline bool codec_is_identity(Codec64 c) { return c.flip == 0 && c.fmask == 0; }

// Which global accesses of a kernel apply the codec.  A sort made of several
// kernels encodes at its first kernel's loads and decodes at its last
// kernel's stores; the kernels in between move keys of the sorting domain
// unchanged, with no codec arithmetic.  CX_BOTH is a kernel that is the whole
// sort; an identity codec always takes CX_NONE.
enum : int { CX_NONE = 0, CX_ENC = 1, CX_DEC = 2, CX_BOTH = 3 };

template <int CX, class C = Codec>
struct KeyIO {
  C c;
  template <class T>
  __device__ __forceinline__ T enc(T x) const {
    if constexpr ((CX & CX_ENC) != 0) return c.enc(x);
    return x;
  }
  template <class T>
  __device__ __forceinline__ T dec(T y) const {
    if constexpr ((CX & CX_DEC) != 0) return c.dec(y);
    return y;
  }
};

// Key types of the C interface (enum bitonic_key_type in bitonic.h).
inline Codec make_codec(int key_type, bool ascending) {
  switch (key_type) {
    case 1: return Codec{ascending ? INT32_MIN : INT32_MAX, 0};          // uint32
    case 2: return Codec{ascending ? 0 : -1, INT32_MAX};                 // float32
    default: return Codec{ascending ? 0 : -1, 0};                        // int32
  }
}

// 8-byte key types (BITONIC_KEY_I64 = 3, U64 = 4, F64 = 5).
inline Codec64 make_codec64(int key_type, bool ascending) {
  switch (key_type) {
    case 4: return Codec64{ascending ? INT64_MIN : INT64_MAX, 0};     // uint64
    case 5: return Codec64{ascending ? 0 : -1, INT64_MAX};            // float64
    default: return Codec64{ascending ? 0 : -1, 0};                   // int64
  }
}

// Pairs with a 4-byte key of key_type (0, 1, 2) and an int32 value.
inline Codec64 make_pair_codec(int key_type, bool ascending) {
  const Codec c = make_codec(key_type, ascending);
  const uint64_t flip = ((uint64_t)(uint32_t)c.flip << 32) | 0x80000000u;
  const uint64_t fmask = (uint64_t)(uint32_t)c.fmask << 32;
  return Codec64{(int64_t)flip, (int64_t)fmask};
}

}  // namespace bitonic
