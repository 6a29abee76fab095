// Kernels of the sort on 8-byte elements: int64 / uint64 / float64 keys, and
// (key, value) pairs of 4-byte words, which travel through the network as one
// 8-byte element (key word high, value word low; see Codec64).
//
// The network, the plan and the tile programs are those of the 4-byte sort
// (sections 3.1-4.2 of the paper): a tile sort of phases 1..L per 2^L-element
// tile in registers and LDS, then for every phase p > L its long strides in
// fused passes over global memory and its last L strides in a tile merge.
// Only the element width changes, and with it the global access pattern:
// threads move one element per register slot with lanes on consecutive
// elements (8-byte accesses for int64 keys, a 4-byte access into each array
// for pairs), which needs no alignment beyond the element's own.
//
//  wide_tile_kernel<L, KIND, CX, ST>  tile sort (KIND 2) or merge (KIND 3)
//  wide_pass_kernel<F, MIRROR, B, ST> F long-stride steps, one column of
//                                     2^F elements per thread
//
// ST is the storage: Keys64 (one array of 8-byte keys) or Pairs (an array of
// 4-byte keys and an array of int32 values).  Indices >= n are absent
// INT64_MAX sentinels of the sorting domain.
#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

// get/put take an element index; getb/putb take the index times kUnit as a
// 32-bit byte offset, so a uniform base plus a lane offset maps onto the
// scalar-base + vector-offset global addressing form.
struct Keys64 {
  static constexpr uint32_t kUnit = 8;
  int64_t* k;
  __device__ __forceinline__ int64_t get(uint32_t i) const { return k[i]; }
  __device__ __forceinline__ void put(uint32_t i, int64_t x) const { k[i] = x; }
  __device__ __forceinline__ Keys64 at(size_t i) const { return Keys64{k + i}; }
  __device__ __forceinline__ int64_t getb(uint32_t b) const {
    return *reinterpret_cast<const int64_t*>(reinterpret_cast<const char*>(k) + b);
  }
  __device__ __forceinline__ void putb(uint32_t b, int64_t x) const {
    *reinterpret_cast<int64_t*>(reinterpret_cast<char*>(k) + b) = x;
  }
};

struct Pairs {
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
  __device__ __forceinline__ int64_t getb(uint32_t b) const {
    const uint32_t hi = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(k) + b);
    const uint32_t lo = *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(v) + b);
    return (int64_t)(((uint64_t)hi << 32) | lo);
  }
  __device__ __forceinline__ void putb(uint32_t b, int64_t x) const {
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(k) + b) = (int32_t)((uint64_t)x >> 32);
    *reinterpret_cast<int32_t*>(reinterpret_cast<char*>(v) + b) = (int32_t)(uint32_t)(uint64_t)x;
  }
};

// One tile of 2^L elements per workgroup, `valid` of them real.
template <int L, int KIND, int CX, class ST>
__global__ __launch_bounds__(1 << (L - kWideRegLog)) void wide_tile_kernel(ST st, uint32_t n,
                                                                           Codec64 codec) {
  using PR = Prog<L, kWideRegLog, KIND>;
  constexpr int LAST = PR::value.ngroups - 1;
  __shared__ int64_t lds[PR::LDSW];
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
  run_from<PR, 0>(x, lds, threadIdx.x);
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

// F consecutive steps on index bits q+F-1 .. q (the first the mirror step of
// the phase if MIRROR).  Thread g0 + blockIdx.x * 256 + threadIdx.x owns
// column c = g mod 2^q of block b = g / 2^q of 2^(q+F) elements: rows
// rho = 0 .. 2^F-1 at c + rho 2^q within the block, the upper half mirrored
// when MIRROR (row rho holds index (2^F-1-(rho mod 2^(F-1))) 2^q + 2^q-1-c).
// Consecutive threads own consecutive columns, so every row access is
// coalesced.
// BOUNDED == false: the whole block lies below n and nothing is checked;
// since 256 divides 2^q a workgroup stays inside one block, so a row's
// address is a workgroup-uniform row start plus the lane's column (or its
// mirror image), which keeps few vector registers live.
// BOUNDED == true: indices >= n read as sentinels and are not stored.
template <int F, bool MIRROR, bool BOUNDED, class ST>
__global__ __launch_bounds__(256) void wide_pass_kernel(ST st, uint32_t n, int q, uint32_t g0) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  int64_t x[ROWS];
  if constexpr (!BOUNDED) {
    const uint32_t gw = g0 + blockIdx.x * 256u;                // uniform
    const size_t bs = (size_t)(gw >> q) << (q + F);             // uniform block start
    const uint32_t col = (gw + threadIdx.x) & ((1u << q) - 1u);
    const uint32_t off = col * ST::kUnit;                       // byte offsets, < 2^(q+3)
    const uint32_t moff = (((1u << q) - 1u) - col) * ST::kUnit;
    auto row_of = [&](int rho) -> uint32_t {                    // uniform row
      return (MIRROR && (rho & TOP)) ? (uint32_t)(ROWS - 1 - (rho & (TOP - 1))) : (uint32_t)rho;
    };
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool mir = MIRROR && (RHO & TOP);
      x[RHO] = st.at(bs + ((size_t)row_of(RHO) << q)).getb(mir ? moff : off);
    });
    __builtin_amdgcn_sched_barrier(0);
    pass_steps<F, MIRROR, 1>(x);
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool mir = MIRROR && (RHO & TOP);
      st.at(bs + ((size_t)row_of(RHO) << q)).putb(mir ? moff : off, x[RHO]);
      __builtin_amdgcn_sched_barrier(0);
    });
  } else {
    const uint32_t g = g0 + blockIdx.x * 256u + threadIdx.x;
    const uint32_t base = (g & ((1u << q) - 1u)) | ((g >> q) << (q + F));
    if (base >= n) return;  // every element of the thread is past n
    const uint32_t span = (1u << (q + F)) - 1u;
    auto row = [&](int rho) -> uint32_t {
      if (MIRROR && (rho & TOP)) return base ^ span ^ ((uint32_t)(rho & (TOP - 1)) << q);
      return base | ((uint32_t)rho << q);
    };
    static_for<0, ROWS>([&](auto RHO) {
      const uint32_t i = row(RHO);
      x[RHO] = i < n ? st.get(i) : kPad64;
    });
    pass_steps<F, MIRROR, 1>(x);
    static_for<0, ROWS>([&](auto RHO) {
      const uint32_t i = row(RHO);
      if (i < n) st.put(i, x[RHO]);
    });
  }
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

template <int F, bool MIRROR, class ST>
static void launch_wide_pass_FM(ST st, uint32_t n, int q, hipStream_t s) {
  // 2^q threads per 2^(q+F) block: blocks wholly below n take the unchecked
  // kernel, the block that straddles n (if any) the checked one
  const uint64_t full = ((uint64_t)n >> (q + F)) << q;   // a multiple of 256 (q >= 8)
  const uint64_t blocks = ((uint64_t)n + (1ull << (q + F)) - 1) >> (q + F);
  const uint64_t total = blocks << q;
  if (full > 0)
    wide_pass_kernel<F, MIRROR, false, ST><<<(uint32_t)(full / 256), 256, 0, s>>>(st, n, q, 0u);
  if (total > full)
    wide_pass_kernel<F, MIRROR, true, ST><<<(uint32_t)((total - full + 255) / 256), 256, 0, s>>>(
        st, n, q, (uint32_t)full);
}

template <int F, class ST>
static void launch_wide_pass_F(bool mirror, ST st, uint32_t n, int q, hipStream_t s) {
  if (mirror)
    launch_wide_pass_FM<F, true>(st, n, q, s);
  else
    launch_wide_pass_FM<F, false>(st, n, q, s);
}

template <class ST>
static void launch_wide_pass_st(int f, bool mirror, ST st, uint32_t n, int q, hipStream_t s) {
  switch (f) {
    case 1: launch_wide_pass_F<1>(mirror, st, n, q, s); break;
    case 2: launch_wide_pass_F<2>(mirror, st, n, q, s); break;
    case 3: launch_wide_pass_F<3>(mirror, st, n, q, s); break;
    case 4: launch_wide_pass_F<4>(mirror, st, n, q, s); break;
    case 5: launch_wide_pass_F<5>(mirror, st, n, q, s); break;
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

void launch_wide_pass(int f, bool mirror, int64_t* keys64, int32_t* keys32, int32_t* values,
                      uint32_t n, int q, hipStream_t s) {
  if (values)
    launch_wide_pass_st(f, mirror, Pairs{keys32, values}, n, q, s);
  else
    launch_wide_pass_st(f, mirror, Keys64{keys64}, n, q, s);
}

}  // namespace bitonic
