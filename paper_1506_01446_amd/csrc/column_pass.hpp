// One-column fused passes over global memory, shared by the sorts of 4-byte
// keys (for 6 to 8 fused steps) and of 8-byte elements (any number), and the
// storage types they read and write.
//
// A storage type names where the elements of a sort live: Keys32 (an array
// of 4-byte keys), Keys64 (an array of 8-byte keys) or Pairs (an array of
// 4-byte keys and an array of int32 values, moving as one 8-byte element:
// key word high, value word low).  E is the element type in registers and
// kPadE the sentinel of the sorting domain for indices >= n.
#pragma once

#include <type_traits>

#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

// get/put take an element index; getb/putb take the index times kUnit as a
// byte offset, 32-bit wherever it fits (pass_offset_bits), so a uniform base
// plus a lane offset maps onto the scalar-base + vector-offset global
// addressing form.
struct Keys32 {
  using E = int32_t;
  static constexpr E kPadE = kPad;
  static constexpr uint32_t kUnit = 4;
  int32_t* k;
  __device__ __forceinline__ int32_t get(uint32_t i) const { return k[i]; }
  __device__ __forceinline__ void put(uint32_t i, int32_t x) const { k[i] = x; }
  __device__ __forceinline__ Keys32 at(size_t i) const { return Keys32{k + i}; }
  template <class O>
  __device__ __forceinline__ int32_t getb(O b) const {
    return *reinterpret_cast<const int32_t*>(reinterpret_cast<const char*>(k) + b);
  }
  template <class O>
  __device__ __forceinline__ void putb(O b, int32_t x) const {
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(k) + b) = x;
  }
};

struct Keys64 {
  using E = int64_t;
  static constexpr E kPadE = kPad64;
  static constexpr uint32_t kUnit = 8;
  int64_t* k;
  __device__ __forceinline__ int64_t get(uint32_t i) const { return k[i]; }
  __device__ __forceinline__ void put(uint32_t i, int64_t x) const { k[i] = x; }
  __device__ __forceinline__ Keys64 at(size_t i) const { return Keys64{k + i}; }
  template <class O>
  __device__ __forceinline__ int64_t getb(O b) const {
    return *reinterpret_cast<const int64_t*>(reinterpret_cast<const char*>(k) + b);
  }
  template <class O>
  __device__ __forceinline__ void putb(O b, int64_t x) const {
    *reinterpret_cast<int64_t*>(reinterpret_cast<char*>(k) + b) = x;
  }
};

struct Pairs {
  using E = int64_t;
  static constexpr E kPadE = kPad64;
  int32_t* k;
  int32_t* v;
  __device__ __forceinline__ int64_t get(uint32_t i) const {
    return (int64_t)(((uint64_t)(uint32_t)k[i] << 32) | (uint32_t)v[i]);
  }
  __device__ __forceinline__ void put(uint32_t i, int64_t x) const {
    k[i] = (int32_t)((uint64_t)x >> 32);
    v[i] = (int32_t)(uint32_t)(uint64_t)x;
  }
  __device__ __forceinline__ Pairs at(size_t i) const { return Pairs{k + i, v + i}; }
  static constexpr uint32_t kUnit = 4;
  template <class O>
  __device__ __forceinline__ int64_t getb(O b) const {
    const uint32_t hi = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(k) + b);
    const uint32_t lo = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(v) + b);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  }
  template <class O>
  __device__ __forceinline__ void putb(O b, int64_t x) const {
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(k) + b) = (int32_t)((uint64_t)x >> 32);
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(v) + b) = (int32_t)(uint32_t)(uint64_t)x;
  }
};

// F consecutive steps on index bits q+F-1 .. q (the first the mirror step of
// the phase if MIRROR).  Thread g = g0 + blockIdx.x * 256 + threadIdx.x owns
// column c = g mod 2^q of block b = g / 2^q of 2^(q+F) elements: rows
// rho = 0 .. 2^F-1 at c + rho 2^q within the block, the upper half mirrored
// when MIRROR (row rho holds index (2^F-1-(rho mod 2^(F-1))) 2^q + 2^q-1-c).
// Consecutive threads own consecutive columns, so every row access is
// coalesced.  Since 256 divides 2^q a workgroup stays inside one block, so a
// row's address is a workgroup-uniform row start plus the lane's column (or
// its mirror image) as a byte offset (32-bit wherever it fits), which keeps few vector
// registers live.  BOUNDED == false: the whole block lies below n and nothing
// is checked.  BOUNDED == true: the workgroups of blocks wholly below n run
// as unchecked, those of the block that straddles n read indices >= n as
// sentinels and do not store them, so one launch covers any n.  OFF64: the lane byte offsets are formed in 64 bits, for rows of
// 2^q elements of kUnit bytes that span more than 2^32 bytes (8-byte
// elements at q = 30; see column_pass_offset_bits).
template <int F, bool MIRROR, bool BOUNDED, class ST, bool OFF64 = false>
__global__ __launch_bounds__(256) void column_pass_kernel(ST st, uint32_t n, int q, uint32_t g0) {
  using E = typename ST::E;
  using Off = std::conditional_t<OFF64, uint64_t, uint32_t>;
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  E x[ROWS];
  const uint32_t gw = g0 + blockIdx.x * 256u;                // uniform
  const uint32_t bs = (gw >> q) << (q + F);                   // uniform block start
  const uint32_t col = (gw + threadIdx.x) & ((1u << q) - 1u);
  const uint32_t mcol = ((1u << q) - 1u) - col;
  // uniform: the block lies wholly below n (always, unless BOUNDED)
  const bool whole = !BOUNDED || (uint64_t)bs + (1ull << (q + F)) <= (uint64_t)n;
  // the thread's lowest index is bs + col; its mirrored rows lie higher
  if (BOUNDED && !whole && bs + col >= n) return;
  const Off off = (Off)col * ST::kUnit;                       // byte offsets, < 2^q kUnit
  const Off moff = (Off)mcol * ST::kUnit;
  auto row_of = [&](int rho) -> uint32_t {                    // uniform row
    return (MIRROR && (rho & TOP)) ? (uint32_t)(ROWS - 1 - (rho & (TOP - 1))) : (uint32_t)rho;
  };
  auto load_rows = [&](auto CHECK) {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool mir = MIRROR && (RHO & TOP);
      const uint32_t r0 = bs + (row_of(RHO) << q);            // uniform
      if constexpr (decltype(CHECK)::value) {
        x[RHO] = r0 + (mir ? mcol : col) < n ? st.at(r0).getb(mir ? moff : off) : ST::kPadE;
      } else {
        x[RHO] = st.at(r0).getb(mir ? moff : off);
      }
    });
  };
  if (whole)
    load_rows(std::false_type{});
  else if constexpr (BOUNDED)
    load_rows(std::true_type{});
  __builtin_amdgcn_sched_barrier(0);
  pass_steps<F, MIRROR, 1>(x);
  __builtin_amdgcn_sched_barrier(0);
  // 4-byte keys: the stores take their row starts from an opaque copy of the
  // block start, so the loads' 2^F row addresses (64-bit scalar pairs) die at
  // the loads instead of living across the steps, where from 64 of them on
  // they overflow the scalar registers and spill to vector lanes (seven-step
  // passes 24-25 -> 22-23 us at n = 2^24).  The 8-byte passes measured slower
  // this way (more vector registers at the same occupancy) and keep theirs.
  uint32_t bs_st = bs;
  if constexpr (sizeof(E) == 4) asm volatile("" : "+s"(bs_st));
  auto store_rows = [&](auto CHECK) {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool mir = MIRROR && (RHO & TOP);
      const uint32_t r0 = bs_st + (row_of(RHO) << q);
      if (!decltype(CHECK)::value || r0 + (mir ? mcol : col) < n)
        st.at(r0).putb(mir ? moff : off, x[RHO]);
      __builtin_amdgcn_sched_barrier(0);
    });
  };
  if (whole)
    store_rows(std::false_type{});
  else if constexpr (BOUNDED)
    store_rows(std::true_type{});
}

template <int F, bool MIRROR, class ST, bool OFF64>
static void launch_column_pass_FMO(ST st, uint32_t n, int q, hipStream_t s) {
  // 2^q threads per 2^(q+F) block (a multiple of 256, q >= 8): when every
  // block lies below n the unchecked kernel, else one launch of the checked
  // one, whose workgroups of whole blocks run unchecked
  const uint64_t full = ((uint64_t)n >> (q + F)) << q;
  const uint64_t blocks = ((uint64_t)n + (1ull << (q + F)) - 1) >> (q + F);
  const uint64_t total = blocks << q;
  if (total == full)
    column_pass_kernel<F, MIRROR, false, ST, OFF64><<<(uint32_t)(full / 256), 256, 0, s>>>(
        st, n, q, 0u);
  else
    column_pass_kernel<F, MIRROR, true, ST, OFF64><<<(uint32_t)(total / 256), 256, 0, s>>>(
        st, n, q, 0u);
}

template <int F, bool MIRROR, class ST>
static void launch_column_pass_FM(ST st, uint32_t n, int q, hipStream_t s) {
  // 64-bit offsets only where column_pass_offset_bits asks for them (one-step
  // passes of 8-byte elements), so only those are instantiated
  if constexpr (F == 1 && ST::kUnit > 4) {
    if (column_pass_offset_bits(ST::kUnit, F, q) > 32) {
      launch_column_pass_FMO<F, MIRROR, ST, true>(st, n, q, s);
      return;
    }
  }
  launch_column_pass_FMO<F, MIRROR, ST, false>(st, n, q, s);
}

template <int F, class ST>
static void launch_column_pass_F(bool mirror, ST st, uint32_t n, int q, hipStream_t s) {
  if (mirror)
    launch_column_pass_FM<F, true>(st, n, q, s);
  else
    launch_column_pass_FM<F, false>(st, n, q, s);
}

}  // namespace bitonic

namespace bitonic {

// F = FR + G steps on index bits q+F-1 .. q of 4-byte keys with every column
// of a 2^(q+F) block split over 2^G neighbouring lanes of 2^FR keys each, so
// that the steps on the top G row bits are cross-lane compare-exchanges
// (DPP) and the other FR run in registers: passes of more steps than one
// thread's registers hold (up to 10 with 2^8 keys per lane), one HBM round
// trip instead of two.  Thread g = blockIdx.x * 256 + threadIdx.x is lane
// s = g mod 2^G of column c = (g / 2^G) mod 2^q of block g / 2^(q+G), and
// holds rows s 2^FR .. s 2^FR + 2^FR - 1 of column c in ascending order.
// With MIRROR the upper half of a column's lanes hold the mirrored rows:
// lane s >= 2^(G-1) holds rows R_s .. R_s + 2^FR - 1 of column 2^q-1-c,
// R_s = 2^F - (s - 2^(G-1) + 1) 2^FR, again ascending, so the mirror step
// pairs register j of lane s with register 2^FR-1-j of lane s XOR 2^(G-1),
// and in every later step the lower register of a pair holds the lower
// index.  Lane byte offsets below 2^(q+F+2) <= 2^32.  The last block may
// end past n (virtual padding): its workgroups load the keys at indices
// n and up as the sentinel and do not store them (exec-masked accesses), so
// every block start is below n and every index below 2^31.  A wave's access
// to one register row is two (G = 1) or four (G = 2) runs of consecutive
// keys.
template <int FR, int G, bool MIRROR>
__global__ __launch_bounds__(256) void column_lanes_pass_kernel(int32_t* __restrict__ keys, int q,
                                                                uint32_t n) {
  constexpr int F = FR + G;
  constexpr int M = 1 << FR;
  constexpr uint32_t SUBS = 1u << G;
  constexpr uint32_t HALF = SUBS >> 1;
  static_assert(G >= 1 && G <= 2, "one or two lane bits per column");
  int32_t x[M];
  const uint32_t gw = blockIdx.x * 256u;                        // uniform
  const uint32_t bs = (gw >> (q + G)) << (q + F);               // uniform block start
  const uint32_t t = (gw + threadIdx.x) & ((1u << (q + G)) - 1u);
  const uint32_t s = t & (SUBS - 1u);
  const uint32_t col = t >> G;
  const bool upper = MIRROR && s >= HALF;
  const uint32_t colx = upper ? ((1u << q) - 1u) - col : col;
  const uint32_t row0 = upper ? (1u << F) - (s - HALF + 1u) * (uint32_t)M : s * (uint32_t)M;
  const uint32_t off = ((row0 << q) + colx) * 4u;               // lane byte offset
  const bool whole = bs + (1u << (q + F)) <= n;                 // uniform
  if (whole) {
    static_for<0, M>([&](auto J) {
      const uint32_t r0 = bs + ((uint32_t)J << q);              // uniform row start
      x[J] = Keys32{keys}.at(r0).getb(off);
    });
  } else {
    static_for<0, M>([&](auto J) {
      const uint32_t r0 = bs + ((uint32_t)J << q);
      x[J] = r0 + (off >> 2) < n ? Keys32{keys}.at(r0).getb(off) : kPad;
    });
  }
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (MIRROR) {
    // the lower half of the column's lanes keeps the minimum of each pair
    const int32_t c = upper ? INT32_MAX : INT32_MIN;
    static_for<0, M / 2>([&](auto J) {
      constexpr int j = J;
      constexpr int jj = M - 1 - j;
      const int32_t pa = lane_xor<HALF>(x[jj]);
      const int32_t pb = lane_xor<HALF>(x[j]);
      x[j] = keep_of_pair(x[j], pa, c);
      x[jj] = keep_of_pair(x[jj], pb, c);
    });
  }
  // half-cleaners on the remaining lane bits, highest first: the lane with
  // the lower rows keeps the minimum (in the mirrored half, the lane whose
  // bit is set)
  constexpr int NL = MIRROR ? G - 1 : G;
  static_for<0, NL>([&](auto I) {
    constexpr int b = NL - 1 - I;
    const bool bit = ((s >> b) & 1u) != 0;
    const int32_t c = (upper ? !bit : bit) ? INT32_MAX : INT32_MIN;
    static_for<0, M>([&](auto J) { x[J] = lane_pair_step<(1u << b)>(x[J], c); });
  });
  pass_steps<FR, false, 1>(x);
  __builtin_amdgcn_sched_barrier(0);
  // row starts for the stores from an opaque copy of the block start (see
  // column_pass_kernel)
  uint32_t bs_st = bs;
  asm volatile("" : "+s"(bs_st));
  if (whole) {
    static_for<0, M>([&](auto J) {
      const uint32_t r0 = bs_st + ((uint32_t)J << q);
      Keys32{keys}.at(r0).putb(off, x[J]);
      __builtin_amdgcn_sched_barrier(0);
    });
  } else {
    static_for<0, M>([&](auto J) {
      const uint32_t r0 = bs_st + ((uint32_t)J << q);
      if (r0 + (off >> 2) < n) Keys32{keys}.at(r0).putb(off, x[J]);
    });
  }
}

// F = FR + 2 steps on index bits q+F-1 .. q of 4-byte keys with every
// column of a 2^(q+F) block spread over the four waves of a workgroup: wave
// w holds rows w 2^FR .. (w+1) 2^FR - 1 of 64 consecutive columns, one key
// per lane and row, so a wave's access to a row is one 256-byte run (the
// lane passes, whose lanes split a column, touch two or four shorter runs).
// With MIRROR the upper two waves hold the mirrored rows of the mirrored
// columns (rows R_w .. R_w + 2^FR - 1 of column 2^q-1-c, R_w = 2^F -
// (w - 1) 2^FR) in descending order, so that register j of the four waves
// holds the four rows one compare-exchange group of the top two row bits
// needs.  Those two steps go through LDS in chunks of C registers (two
// buffers, two barriers per chunk): every wave writes its registers of the
// chunk, takes a quarter of the slots, performs both steps on the four keys
// of each, writes them back, and reads its own again.  The other FR steps
// run in registers; the mirrored waves, whose rows descend, hold their keys
// complemented meanwhile (~ reverses the signed order), so the same
// ascending steps serve every wave.  Whole blocks only (wave_pass_fits).
template <int FR, bool MIRROR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, FR >= 8 ? 1 : 2)))
void column_waves_pass_kernel(int32_t* __restrict__ keys, int q) {
  constexpr int F = FR + 2;
  constexpr int M = 1 << FR;
  constexpr int C = 32;  // registers per chunk
  static_assert(M % C == 0 && C % 4 == 0, "whole chunks, quarters of a chunk");
  __shared__ int32_t xch[2][4][C][64];
  int32_t x[M];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const uint32_t g = blockIdx.x;  // one workgroup per 64 columns of a block
  const uint32_t bs = (g >> (q - 6)) << (q + F);  // uniform block start
  const uint32_t c = ((g & ((1u << (q - 6)) - 1u)) << 6) + lane;
  const bool upper = MIRROR && w >= 2u;
  const uint32_t colx = upper ? ((1u << q) - 1u) - c : c;
  // row of register j: row0 + j, or (mirrored waves) row0 - j
  const uint32_t row0 = upper ? (1u << F) - (w - 1u) * (uint32_t)M + (uint32_t)(M - 1)
                              : w * (uint32_t)M;
  const uint32_t off = colx * 4u;  // lane byte offset inside a row
  auto row_of = [&](uint32_t j) { return upper ? row0 - j : row0 + j; };  // wave-uniform
  const int32_t flip = upper ? -1 : 0;  // complement of the mirrored waves' keys
  static_for<0, M>([&](auto J) {
    const uint32_t r0 = bs + (row_of(J) << q);
    x[J] = Keys32{keys}.at(r0).getb(off);
  });
  static_for<0, M / C>([&](auto K) {
    constexpr int b = K & 1;
    static_for<0, C>([&](auto J) { xch[b][w][J][lane] = x[K * C + J]; });
    __syncthreads();
    static_for<0, C / 4>([&](auto I) {
      const uint32_t j = w * (C / 4) + I;
      int32_t a0 = xch[b][0][j][lane], a1 = xch[b][1][j][lane];
      int32_t a2 = xch[b][2][j][lane], a3 = xch[b][3][j][lane];
      cmpx(a0, a2);  // the mirror step, or the step on the top row bit
      cmpx(a1, a3);
      cmpx(a0, a1);
      if constexpr (MIRROR)
        cmpx(a3, a2);  // wave 3 holds the lower rows of the mirrored half
      else
        cmpx(a2, a3);
      xch[b][0][j][lane] = a0;
      xch[b][1][j][lane] = a1;
      xch[b][2][j][lane] = a2;
      xch[b][3][j][lane] = a3;
    });
    __syncthreads();
    static_for<0, C>([&](auto J) { x[K * C + J] = xch[b][w][J][lane] ^ flip; });
  });
  pass_steps<FR, false, 1>(x);
  __builtin_amdgcn_sched_barrier(0);
  uint32_t bs_st = bs;
  asm volatile("" : "+s"(bs_st));
  static_for<0, M>([&](auto J) {
    const uint32_t r0 = bs_st + (row_of(J) << q);
    Keys32{keys}.at(r0).putb(off, x[J] ^ flip);
    __builtin_amdgcn_sched_barrier(0);
  });
}

template <int FR>
static void launch_column_waves_F(bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  const uint32_t blocks = n >> (FR + 8);  // one workgroup per 64 columns x 2^(FR+2) rows
  if (mirror)
    column_waves_pass_kernel<FR, true><<<blocks, 256, 0, st>>>(keys, q);
  else
    column_waves_pass_kernel<FR, false><<<blocks, 256, 0, st>>>(keys, q);
}

template <int FR, int G>
static void launch_column_lanes_FG(bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  // the 2^(q+F)-key blocks that start below n, 2^(q+G) threads each, 256
  // per workgroup
  constexpr int F = FR + G;
  const uint32_t nblocks = (uint32_t)(((uint64_t)n + (1u << (q + F)) - 1u) >> (q + F));
  const uint32_t blocks = nblocks << (q + G - 8);
  if (mirror)
    column_lanes_pass_kernel<FR, G, true><<<blocks, 256, 0, st>>>(keys, q, n);
  else
    column_lanes_pass_kernel<FR, G, false><<<blocks, 256, 0, st>>>(keys, q, n);
}

}  // namespace bitonic
