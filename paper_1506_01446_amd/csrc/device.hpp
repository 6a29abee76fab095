// Device-side building blocks shared by the plain and segmented kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <climits>

#include <type_traits>

#include "codec.hpp"
#include "program.hpp"

namespace bitonic {

// Sentinel in the sorting domain.  Stored keys are mapped by a Codec to the
// sorting domain, where they are sorted as signed int32 ascending, so the
// absent padding keys are always INT32_MAX there.
constexpr int32_t kPad = 0x7FFFFFFF;

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// Sentinel of the 8-byte sorting domain (int64 keys and packed pairs).
constexpr int64_t kPad64 = 0x7FFFFFFFFFFFFFFFll;

// Compare-exchange: a takes the minimum, b the maximum.
__device__ __forceinline__ void cmpx(int32_t& a, int32_t& b) {
  const int32_t lo = min(a, b);
  const int32_t hi = max(a, b);
  a = lo;
  b = hi;
}

__device__ __forceinline__ void cmpx(int64_t& a, int64_t& b) {
  const bool sw = b < a;
  const int64_t lo = sw ? b : a;
  const int64_t hi = sw ? a : b;
  a = lo;
  b = hi;
}

// Spread the low bits of t over the set bits of MASK (lowest first).
template <uint32_t MASK>
__device__ __forceinline__ uint32_t deposit(uint32_t t) {
  uint32_t out = 0;
  static_for<0, 32>([&](auto B) {
    constexpr int b = B;
    if constexpr ((MASK >> b) & 1u) {
      constexpr int k = __builtin_popcount(MASK & ((1u << b) - 1u));
      out |= ((t >> k) & 1u) << b;
    }
  });
  return out;
}

// Program of a tile kernel, as a type.
template <int L_, int R_LOG_, int KIND_>
struct Prog {
  static constexpr int L = L_;
  static constexpr int RL = R_LOG_;
  static constexpr int R = 1 << R_LOG_;
  static constexpr int NT = 1 << (L_ - R_LOG_);
  static constexpr int T = 1 << L_;
  static constexpr uint32_t LDSW = lds_words(L_, R_LOG_);  // padded LDS words of a tile
  static constexpr bool VEC = kind_is_vector(KIND_);  // 16-byte vector global I/O allowed
  // Recompute each layout's thread base at its regroup (fewer registers,
  // more ALU); used by the segment kernels, which run several programs in
  // one kernel.  (The single-array tile kernels keep the bases: 59 VGPRs
  // for the 2^14-key sort, 114 for the 2^15-key merge loop, both within the
  // 128 their workgroup sizes allow.)
  static constexpr bool LEAN = kind_is_lean(KIND_);
  static constexpr Program value = make_program(L_, R_LOG_, KIND_);
  static_assert(value.ngroups <= kMaxGroups, "program too long");
};

// v's value in lane (this lane XOR M) of the wave: DPP moves inside rows of
// 16 lanes for M < 16, the swizzle that reverses groups of 32 lanes for
// M = 31, a lane permute for M = 63.
template <uint32_t M>
__device__ __forceinline__ int32_t lane_xor(int32_t v) {
  if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm 1032
  else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // 2301
  else if constexpr (M == 3) return __builtin_amdgcn_mov_dpp(v, 0x1B, 0xF, 0xF, false);  // 3210
  else if constexpr (M == 7) return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  else if constexpr (M == 15) return __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, false);  // row_mirror
  else if constexpr (M == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);   // row_ror:8
  else if constexpr (M == 4) return lane_xor<3>(lane_xor<7>(v));
  else if constexpr (M == 31) return __builtin_amdgcn_ds_swizzle(v, 0x7C1F);  // xor 31 in 32 lanes
  else if constexpr (M == 63) {
    const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return __builtin_amdgcn_ds_bpermute((int)((lane ^ 63u) << 2), v);
  } else static_assert(M == 1, "lane exchange pattern not provided");
  return v;
}

// The key a lane keeps from the pair (a, b): the maximum where c = INT32_MAX
// (the upper end of the pair), the minimum where c = INT32_MIN; one v_med3.
__device__ __forceinline__ int32_t keep_of_pair(int32_t a, int32_t b, int32_t c) {
  return max(min(a, b), min(max(a, b), c));
}

// A lane step of one register with itself (partner: the same slot of lane
// XOR M).  For M = 16 and 32 the gfx950 permlane swaps of the register with
// itself leave the pair's two keys in every lane (the swap's two results), in
// either order, which is all keep_of_pair needs.
template <uint32_t M>
__device__ __forceinline__ int32_t lane_pair_step(int32_t x, int32_t c) {
  if constexpr (M == 16) {
    const auto s = __builtin_amdgcn_permlane16_swap((uint32_t)x, (uint32_t)x, false, false);
    return keep_of_pair((int32_t)s[0], (int32_t)s[1], c);
  } else if constexpr (M == 32) {
    const auto s = __builtin_amdgcn_permlane32_swap((uint32_t)x, (uint32_t)x, false, false);
    return keep_of_pair((int32_t)s[0], (int32_t)s[1], c);
  } else {
    return keep_of_pair(x, lane_xor<M>(x), c);
  }
}

// All compare-exchange steps of group G on the registers.
template <class PR, int G, class E>
__device__ __forceinline__ void group_steps(E (&x)[PR::R]) {
  constexpr Group gr = PR::value.g[G];
  static_for<0, gr.nsteps>([&](auto S) {
    constexpr uint32_t D = gr.d[S];
    if constexpr (step_lane(D) == 0) {
      static_for<0, PR::R>([&](auto J) {
        constexpr uint32_t j = J;
        constexpr uint32_t jj = j ^ D;
        if constexpr (j < jj) {
          if constexpr (slot_is_lower(gr, j, D)) {
            cmpx(x[j], x[jj]);
          } else {
            cmpx(x[jj], x[j]);
          }
        }
      });
    } else {
      // lane step: every slot meets a slot of lane (lane XOR M); the lane
      // whose bit highbit(M) is set holds the upper end of all its pairs
      static_assert(sizeof(E) == 4, "lane steps move 4-byte keys");
      constexpr uint32_t M = step_lane(D);
      constexpr uint32_t DR = step_reg(D);
      const uint32_t lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
      const int32_t c = ((lane >> highbit(M)) & 1u) ? INT32_MAX : INT32_MIN;
      static_for<0, PR::R>([&](auto J) {
        constexpr uint32_t j = J;
        constexpr uint32_t jj = j ^ DR;
        if constexpr (DR == 0) {
          x[j] = lane_pair_step<M>(x[j], c);
        } else if constexpr (j < jj) {
          const int32_t pa = lane_xor<M>(x[jj]);
          const int32_t pb = lane_xor<M>(x[j]);
          x[j] = keep_of_pair(x[j], pa, c);
          x[jj] = keep_of_pair(x[jj], pb, c);
        }
      });
    }
  });
}

// LDS position of the thread part of a layout's slots: P(base), and for the
// mirrored half of a virtual layout P(base ^ (mirror mask on thread bits)).
template <class PR, int G>
struct LdsBase {
  uint32_t plain, mirrored;
  __device__ __forceinline__ explicit LdsBase(uint32_t tid) {
    constexpr Group gr = PR::value.g[G];
    const uint32_t b = deposit<free_mask(gr, PR::L)>(tid);
    plain = lds_pad(b, PR::RL);
    if constexpr (gr.vmirror > 0)
      mirrored = lds_pad(b ^ (mirror_mask(gr) & free_mask(gr, PR::L)), PR::RL);
    else
      mirrored = plain;
  }
  template <uint32_t J>
  __device__ __forceinline__ uint32_t at() const {
    constexpr Group gr = PR::value.g[G];
    constexpr uint32_t o = lds_pad(real_off(gr, J), PR::RL);
    return (slot_mirrored(gr, J) ? mirrored : plain) + o;
  }
};

// Orders the LDS accesses of the lanes of one wave: a wave's LDS
// instructions execute in order, so only the compiler must be kept from
// moving accesses across (fences at wavefront scope and a wave barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronisation between the LDS writes and reads of the regroup from group
// GA to GB: a workgroup barrier, or only a wave-level ordering when the
// regroup keeps every key inside its wave (regroup_in_wave).
template <class PR, int GA, int GB>
__device__ __forceinline__ void regroup_sync() {
  if constexpr (regroup_in_wave(PR::value.g[GA], PR::value.g[GB], PR::L))
    wave_sync();
  else
    __syncthreads();
}

// Before a program's first regroup writes LDS, the previous user of the LDS
// (the previous tile of a kernel that loops over tiles) must be done with
// it.  Later regroups need no such wait: a regroup writes each key at the
// position of its real index in the layout it starts from, exactly where the
// previous regroup read it, and in one layout the waves hold disjoint sets
// of indices, so no wave overwrites a position another wave may still read.
template <int GA>
__device__ __forceinline__ void regroup_enter() {
  if constexpr (GA == 0) __syncthreads();
}

// Move the registers from the layout of group GA to that of group GB
// through LDS (each key to the padded position of its real index).
template <class PR, int GA, int GB, class E>
__device__ __forceinline__ void regroup(E (&x)[PR::R], E* lds, uint32_t tid) {
  if constexpr (PR::LEAN) asm volatile("" : "+v"(tid));
  const LdsBase<PR, GA> a(tid);
  const LdsBase<PR, GB> b(tid);
  regroup_enter<GA>();
  static_for<0, PR::R>([&](auto J) { lds[a.template at<J>()] = x[J]; });
  regroup_sync<PR, GA, GB>();
  static_for<0, PR::R>([&](auto J) { x[J] = lds[b.template at<J>()]; });
}

template <class PR, int G, class E>
__device__ __forceinline__ void run_from(E (&x)[PR::R], E* lds, uint32_t tid) {
  group_steps<PR, G>(x);
  if constexpr (G + 1 < PR::value.ngroups) {
    regroup<PR, G, G + 1>(x, lds, tid);
    run_from<PR, G + 1>(x, lds, tid);
  }
}

// Index of register slot J of a thread whose base index is `base` (layouts
// used for global I/O are never virtual).
template <class PR, int G, uint32_t J>
__device__ __forceinline__ uint32_t slot_index(uint32_t base) {
  constexpr Group gr = PR::value.g[G];
  static_assert(gr.vmirror == 0, "global I/O from a virtual layout");
  return base + goff(gr, J);
}

// Load the thread's keys of a tile in the layout of group G.
// `valid` keys of the tile exist; the rest read as the sentinel.
template <class PR, int G, class CD>
__device__ __forceinline__ void load_tile(int32_t (&x)[PR::R], const int32_t* __restrict__ tile,
                                          uint32_t valid, CD cd, uint32_t tid) {
  constexpr Group gr = PR::value.g[G];
  const uint32_t base = deposit<free_mask(gr, PR::L)>(tid);
  if (valid >= (uint32_t)PR::T) {
    if constexpr (PR::VEC && layout_is_vector4(gr)) {
      static_for<0, PR::R / 4>([&](auto Q) {
        constexpr uint32_t o = goff(gr, 4u * Q);
        const uint32_t i = slot_index<PR, G, 4u * Q>(base);
        const int4 v = *reinterpret_cast<const int4*>(tile + (i & ~3u));
        const int32_t e[4] = {v.x, v.y, v.z, v.w};
        static_for<0, 4>([&](auto C) {
          x[4 * Q + C] = cd.enc(e[(o ^ C) & 3u]);
        });
      });
    } else {
      static_for<0, PR::R>([&](auto J) { x[J] = cd.enc(tile[slot_index<PR, G, J>(base)]); });
    }
  } else {
    static_for<0, PR::R>([&](auto J) {
      const uint32_t i = slot_index<PR, G, J>(base);
      x[J] = i < valid ? cd.enc(tile[i]) : kPad;
    });
  }
}

// Buffer resource over the 2^L keys of a tile starting at `tile`, or an empty
// one (`full` false).  Buffer loads outside the range return zeros and read no
// memory, so a load of "no tile" issues the same instructions as a real one.
// The last word is the gfx9-family resource format for raw 32-bit data.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const int32_t* tile, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(tile), 0, (int)bytes, 0x00020000);
}

// A full tile in the 16-byte layout of group G through a buffer resource.
template <class PR, int G, class CD>
__device__ __forceinline__ void load_tile_rsrc(int32_t (&x)[PR::R], __amdgpu_buffer_rsrc_t rs,
                                               CD cd, uint32_t tid) {
  constexpr Group gr = PR::value.g[G];
  static_assert(PR::VEC && layout_is_vector4(gr), "buffer tile loads need the 16-byte layout");
  const uint32_t base = deposit<free_mask(gr, PR::L)>(tid);
  static_for<0, PR::R / 4>([&](auto Q) {
    constexpr uint32_t o = goff(gr, 4u * Q);
    const uint32_t i = slot_index<PR, G, 4u * Q>(base);
    const int4 v = __builtin_bit_cast(
        int4, __builtin_amdgcn_raw_buffer_load_b128(rs, (i & ~3u) * 4u, 0, 0));
    const int32_t e[4] = {v.x, v.y, v.z, v.w};
    static_for<0, 4>([&](auto C) { x[4 * Q + C] = cd.enc(e[(o ^ C) & 3u]); });
  });
}

template <class PR, int G, class CD>
__device__ __forceinline__ void store_tile(const int32_t (&x)[PR::R], int32_t* __restrict__ tile,
                                           uint32_t valid, CD cd, uint32_t tid) {
  constexpr Group gr = PR::value.g[G];
  const uint32_t base = deposit<free_mask(gr, PR::L)>(tid);
  if (valid >= (uint32_t)PR::T) {
    if constexpr (PR::VEC && layout_is_vector4(gr)) {
      static_for<0, PR::R / 4>([&](auto Q) {
        constexpr uint32_t o = goff(gr, 4u * Q);
        const uint32_t i = slot_index<PR, G, 4u * Q>(base);
        int32_t e[4];
        static_for<0, 4>([&](auto C) { e[(o ^ C) & 3u] = cd.dec(x[4 * Q + C]); });
        *reinterpret_cast<int4*>(tile + (i & ~3u)) = make_int4(e[0], e[1], e[2], e[3]);
      });
    } else {
      static_for<0, PR::R>([&](auto J) { tile[slot_index<PR, G, J>(base)] = cd.dec(x[J]); });
    }
  } else {
    static_for<0, PR::R>([&](auto J) {
      const uint32_t i = slot_index<PR, G, J>(base);
      if (i < valid) tile[i] = cd.dec(x[J]);
    });
  }
}

// Fused long-stride steps on COLS columns x 2^F rows of registers
// x[COLS rho + c]: the mirror step (if MIRROR) on the top row bit, then
// half-cleaners on the remaining row bits, highest first.  Rows of the upper
// half are held mirrored when MIRROR (row rho + 2^(F-1) is the mirror image
// of row rho), so there the lower index of a pair is the row with the bit set.
template <int F, bool MIRROR, int COLS = 4, class E>
__device__ __forceinline__ void pass_steps(E (&x)[COLS << F]) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  if constexpr (MIRROR) {
    static_for<0, TOP>([&](auto RHO) {
      static_for<0, COLS>([&](auto C) { cmpx(x[COLS * RHO + C], x[COLS * (RHO + TOP) + C]); });
    });
  }
  constexpr int NB = MIRROR ? F - 1 : F;
  static_for<0, NB>([&](auto I) {
    constexpr int b = NB - 1 - I;
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      constexpr int partner = rho ^ (1 << b);
      if constexpr (rho < partner) {
        constexpr bool low = !(MIRROR && (rho & TOP));
        static_for<0, COLS>([&](auto C) {
          if constexpr (low) {
            cmpx(x[COLS * rho + C], x[COLS * partner + C]);
          } else {
            cmpx(x[COLS * partner + C], x[COLS * rho + C]);
          }
        });
      }
    });
  });
}

// Sort (KIND 0) or merge (KIND 1) one tile that starts at `tile` and holds
// `valid` real keys.  All threads of the block must call it.  `cd` is a Codec
// or a KeyIO.
template <class PR, class CD>
__device__ __forceinline__ void tile_program(int32_t* __restrict__ tile, uint32_t valid,
                                             CD cd, int32_t* lds, uint32_t tid) {
  int32_t x[PR::R];
  load_tile<PR, 0>(x, tile, valid, cd, tid);
  run_from<PR, 0>(x, lds, tid);
  store_tile<PR, PR::value.ngroups - 1>(x, tile, valid, cd, tid);
}

}  // namespace bitonic
