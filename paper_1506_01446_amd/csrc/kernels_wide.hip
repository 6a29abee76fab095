// Kernels of the sort on 8-byte elements: int64 / uint64 / float64 keys, and
// (key, value) pairs of 4-byte words, which travel through the network as one
// 8-byte element (key word high, value word low; see Codec64).
//
// The network, the plan and the tile programs are those of the 4-byte sort
// (sections 3.1-4.2 of the paper): a tile sort of phases 1..L per 2^L-element
// tile in registers and LDS, then for every phase p > L its long strides in
// fused passes over global memory and its last L strides in a tile merge.
// The element width changes, and with it the register count (16 elements per
// thread), the regroups (high words, then low words, through 4-byte LDS
// words: a 2^13-element tile is an eight-wave workgroup of 34 KiB and four
// share a CU) and the global access pattern:
// threads move one element per register slot with lanes on consecutive
// elements (8-byte accesses for int64 keys, a 4-byte access into each array
// for pairs), which needs no alignment beyond the element's own.
//
//  wide_tile_kernel<L, KIND, CX, ST>  tile sort (KIND 2), merge (KIND 3) or
//                                     phase L (KIND 7: phase t+1 on tiles
//                                     twice the sort's tile)
//  column_pass_kernel<F, MIRROR, B, ST>  F long-stride steps, one column of
//                                        2^F elements per thread (column_pass.hpp)
//  wide_lanes_pass_kernel<FR, G, MIRROR, ST>  F = FR + G = 7, 8 steps, each
//                                        column split over 2^G lanes (as
//                                        column_lanes_pass_kernel)
//
// ST is the storage: Keys64 (one array of 8-byte keys) or Pairs (an array of
// 4-byte keys and an array of int32 values).  Indices >= n are absent
// INT64_MAX sentinels of the sorting domain.
#include "column_pass.hpp"
#include "launch.hpp"
#include "split_regroup.hpp"

namespace bitonic {

// One tile of 2^L elements per workgroup, `valid` of them real.
template <int L, int KIND, int CX, class ST>
__global__ __launch_bounds__(1 << (L - kWideRegLog)) void wide_tile_kernel(ST st, uint32_t n,
                                                                           Codec64 codec) {
  using PR = Prog<L, kWideRegLog, KIND>;
  constexpr int LAST = PR::value.ngroups - 1;
  __shared__ uint32_t lds[PR::LDSW];  // 4-byte words: run_from_split
  const KeyIO<CX, Codec64> cd{codec};
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < (uint32_t)PR::T ? left : (uint32_t)PR::T;
  const bool full = valid == (uint32_t)PR::T;  // uniform
  const ST tile = st.at(t0);
  int64_t x[PR::R];
  {
    constexpr Group gr = PR::value.g[0];
    const uint32_t base = deposit<free_mask(gr, L)>(threadIdx.x);
    if (full) {
      static_for<0, PR::R>([&](auto J) { x[J] = cd.enc(tile.get(slot_index<PR, 0, J>(base))); });
    } else {
      static_for<0, PR::R>([&](auto J) {
        const uint32_t i = slot_index<PR, 0, J>(base);
        x[J] = i < valid ? cd.enc(tile.get(i)) : kPad64;
      });
    }
  }
  run_from_split<PR, 0>(x, lds, threadIdx.x);
  {
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    constexpr Group gr = PR::value.g[LAST];
    const uint32_t base = deposit<free_mask(gr, L)>(tid);
    if (full) {
      static_for<0, PR::R>([&](auto J) { tile.put(slot_index<PR, LAST, J>(base), cd.dec(x[J])); });
    } else {
      static_for<0, PR::R>([&](auto J) {
        const uint32_t i = slot_index<PR, LAST, J>(base);
        if (i < valid) tile.put(i, cd.dec(x[J]));
      });
    }
  }
}

// An 8-byte element's value in lane (this lane XOR M): both words moved.
template <uint32_t M>
__device__ __forceinline__ int64_t lane_xor64(int64_t v) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)lane_xor<M>((int32_t)(uint32_t)u);
  const uint32_t hi = (uint32_t)lane_xor<M>((int32_t)(uint32_t)(u >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The element a lane keeps from the pair (a, b): the larger where `upper`.
__device__ __forceinline__ int64_t keep_of_pair64(int64_t a, int64_t b, bool upper) {
  return (a < b) == upper ? b : a;
}

// F = FR + G long-stride steps of an 8-byte sort with every column of a
// 2^(q+F) block split over 2^G neighbouring lanes of 2^FR elements (the
// layout of column_lanes_pass_kernel: lane s holds rows s 2^FR .. of column
// c, or with MIRROR in the upper half of the lanes the mirrored rows of the
// mirrored column, ascending).  Whole blocks only, lane byte offsets below
// 2^(q+F) kUnit <= 2^32 (wide_lanes_fit).
template <int FR, int G, bool MIRROR, class ST>
__global__ __launch_bounds__(256) void wide_lanes_pass_kernel(ST st, int q) {
  constexpr int F = FR + G;
  constexpr int M = 1 << FR;
  constexpr uint32_t SUBS = 1u << G;
  constexpr uint32_t HALF = SUBS >> 1;
  static_assert(G >= 1 && G <= 2, "one or two lane bits per column");
  int64_t x[M];
  const uint32_t gw = blockIdx.x * 256u;                        // uniform
  const uint32_t bs = (gw >> (q + G)) << (q + F);               // uniform block start
  const uint32_t t = (gw + threadIdx.x) & ((1u << (q + G)) - 1u);
  const uint32_t s = t & (SUBS - 1u);
  const uint32_t col = t >> G;
  const bool upper = MIRROR && s >= HALF;
  const uint32_t colx = upper ? ((1u << q) - 1u) - col : col;
  const uint32_t row0 = upper ? (1u << F) - (s - HALF + 1u) * (uint32_t)M : s * (uint32_t)M;
  const uint32_t off = ((row0 << q) + colx) * ST::kUnit;       // lane byte offset
  static_for<0, M>([&](auto J) {
    const uint32_t r0 = bs + ((uint32_t)J << q);                // uniform row start
    x[J] = st.at(r0).getb(off);
  });
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (MIRROR) {
    static_for<0, M / 2>([&](auto J) {
      constexpr int j = J;
      constexpr int jj = M - 1 - j;
      const int64_t pa = lane_xor64<HALF>(x[jj]);
      const int64_t pb = lane_xor64<HALF>(x[j]);
      x[j] = keep_of_pair64(x[j], pa, upper);
      x[jj] = keep_of_pair64(x[jj], pb, upper);
    });
  }
  constexpr int NL = MIRROR ? G - 1 : G;
  static_for<0, NL>([&](auto I) {
    constexpr int b = NL - 1 - I;
    const bool bit = ((s >> b) & 1u) != 0;
    const bool keep_max = upper ? !bit : bit;
    static_for<0, M>([&](auto J) {
      x[J] = keep_of_pair64(x[J], lane_xor64<(1u << b)>(x[J]), keep_max);
    });
  });
  pass_steps<FR, false, 1>(x);
  __builtin_amdgcn_sched_barrier(0);
  static_for<0, M>([&](auto J) {
    const uint32_t r0 = bs + ((uint32_t)J << q);
    st.at(r0).putb(off, x[J]);
    __builtin_amdgcn_sched_barrier(0);
  });
}

// ---------------------------------------------------------------------------
// launchers

template <int L, class ST>
static void launch_wide_tile_L(int kind, ST st, uint32_t n, Codec64 cd, int cx, hipStream_t s) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kWideRegLog);
  if (codec_is_identity(cd)) cx = CX_NONE;
  if (kind == 0) {
    if (cx == CX_NONE)
      wide_tile_kernel<L, 2, CX_NONE, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
    else if (cx == CX_ENC)
      wide_tile_kernel<L, 2, CX_ENC, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
    else
      wide_tile_kernel<L, 2, CX_BOTH, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
  } else if (cx == CX_NONE) {
    wide_tile_kernel<L, 3, CX_NONE, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
  } else {
    wide_tile_kernel<L, 3, CX_DEC, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
  }
}

template <class ST>
static void launch_wide_tile_st(int L, int kind, ST st, uint32_t n, Codec64 cd, int cx,
                                hipStream_t s) {
  switch (L) {
    case 11: launch_wide_tile_L<11>(kind, st, n, cd, cx, s); break;
    case 12: launch_wide_tile_L<12>(kind, st, n, cd, cx, s); break;
    case 13: launch_wide_tile_L<13>(kind, st, n, cd, cx, s); break;
    default: break;
  }
}

template <int L, class ST>
static void launch_wide_phase_L(ST st, uint32_t n, Codec64 cd, int cx, hipStream_t s) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kWideRegLog);
  if (codec_is_identity(cd)) cx = CX_NONE;
  if (cx == CX_NONE)
    wide_tile_kernel<L, 7, CX_NONE, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
  else
    wide_tile_kernel<L, 7, CX_DEC, ST><<<ntiles, NT, 0, s>>>(st, n, cd);
}

template <class ST>
static void launch_wide_phase_st(int L, ST st, uint32_t n, Codec64 cd, int cx, hipStream_t s) {
  switch (L) {
    case 12: launch_wide_phase_L<12>(st, n, cd, cx, s); break;
    case 13: launch_wide_phase_L<13>(st, n, cd, cx, s); break;
    case 14: launch_wide_phase_L<14>(st, n, cd, cx, s); break;
    default: break;
  }
}

template <int G, class ST>
static void launch_wide_lanes_G(bool mirror, ST st, uint32_t n, int q, hipStream_t s) {
  constexpr int FR = kWideLaneRegLog;
  const uint32_t blocks = n >> (FR + 8);  // n / 2^FR threads, 256 per workgroup
  if (mirror)
    wide_lanes_pass_kernel<FR, G, true, ST><<<blocks, 256, 0, s>>>(st, q);
  else
    wide_lanes_pass_kernel<FR, G, false, ST><<<blocks, 256, 0, s>>>(st, q);
}

template <class ST>
static void launch_wide_pass_st(int f, bool mirror, ST st, uint32_t n, int q, hipStream_t s) {
  if (f > kWideFuseMaxColumn) {  // the planner checked wide_lanes_fit
    if (f == kWideLaneRegLog + 1) launch_wide_lanes_G<1>(mirror, st, n, q, s);
    if (f == kWideLaneRegLog + 2) launch_wide_lanes_G<2>(mirror, st, n, q, s);
    return;
  }
  switch (f) {
    case 1: launch_column_pass_F<1>(mirror, st, n, q, s); break;
    case 2: launch_column_pass_F<2>(mirror, st, n, q, s); break;
    case 3: launch_column_pass_F<3>(mirror, st, n, q, s); break;
    case 4: launch_column_pass_F<4>(mirror, st, n, q, s); break;
    case 5: launch_column_pass_F<5>(mirror, st, n, q, s); break;
    case 6: launch_column_pass_F<6>(mirror, st, n, q, s); break;
    default: break;
  }
}

void launch_wide_tile(int L, int kind, int64_t* keys64, int32_t* keys32, int32_t* values,
                      uint32_t n, Codec64 cd, int cx, hipStream_t s) {
  if (values)
    launch_wide_tile_st(L, kind, Pairs{keys32, values}, n, cd, cx, s);
  else
    launch_wide_tile_st(L, kind, Keys64{keys64}, n, cd, cx, s);
}

void launch_wide_phase(int L, int64_t* keys64, int32_t* keys32, int32_t* values, uint32_t n,
                       Codec64 cd, int cx, hipStream_t s) {
  if (values)
    launch_wide_phase_st(L, Pairs{keys32, values}, n, cd, cx, s);
  else
    launch_wide_phase_st(L, Keys64{keys64}, n, cd, cx, s);
}

void launch_wide_pass(int f, bool mirror, int64_t* keys64, int32_t* keys32, int32_t* values,
                      uint32_t n, int q, hipStream_t s) {
  if (values)
    launch_wide_pass_st(f, mirror, Pairs{keys32, values}, n, q, s);
  else
    launch_wide_pass_st(f, mirror, Keys64{keys64}, n, q, s);
}

}  // namespace bitonic
