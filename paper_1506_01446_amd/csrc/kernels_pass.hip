// The fused long-stride passes of the single-array sort of 4-byte keys.
//
//  global_pass_kernel<F, MIRROR, BOUNDED>  F consecutive steps with strides
//      >= 2^q in one pass over HBM: each thread holds 4 columns x 2^F rows of
//      keys in registers (section 4.2, generalised from 2 steps to F), for
//      F <= 5; wider passes take the one-column kernel (kernels_column.hip).
//
// Passes sit between a sort's first and last kernels, so they move keys of
// the sorting domain (see Codec) unchanged; indices >= n are absent INT32_MAX
// sentinels.
#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

// Keys of thread g: 4 consecutive columns x 2^F rows.  Row rho sits at
// index base | rho << q; with MIRROR the upper half of the rows are the
// mirror images (index XOR (2^(q+F) - 1)), so the first step pairs each key
// with its mirror in the 2^(q+F) block.
template <int F, bool MIRROR, int RHO>
__device__ __forceinline__ uint32_t pass_row_index(uint32_t base, uint32_t span, int q) {
  constexpr int TOP = (1 << F) >> 1;
  if constexpr (MIRROR && (RHO & TOP))
    return base ^ span ^ ((uint32_t)(RHO & (TOP - 1)) << q);
  else
    return base | ((uint32_t)RHO << q);
}

// Row RHO into registers x[4 RHO .. 4 RHO + 3]: one 16-byte load if VEC, else
// key by key with indices >= n read as the sentinel.  Mirrored rows are
// stored in reverse order, so their registers are reversed.
template <int F, bool MIRROR, int RHO, bool VEC>
__device__ __forceinline__ void pass_load_row(int32_t* x, const int32_t* __restrict__ keys,
                                              uint32_t ri, uint32_t n) {
  constexpr bool rev = MIRROR && (RHO & ((1 << F) >> 1));
  if constexpr (VEC) {
    const int4 v = *reinterpret_cast<const int4*>(keys + (ri & ~3u));
    x[4 * RHO + (rev ? 3 : 0)] = v.x;
    x[4 * RHO + (rev ? 2 : 1)] = v.y;
    x[4 * RHO + (rev ? 1 : 2)] = v.z;
    x[4 * RHO + (rev ? 0 : 3)] = v.w;
  } else {
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
      const uint32_t i = ri ^ c;
      x[4 * RHO + c] = i < n ? keys[i] : kPad;
    }
  }
}

template <int F, bool MIRROR, int RHO, bool VEC>
__device__ __forceinline__ void pass_store_row(const int32_t* x, int32_t* __restrict__ keys,
                                               uint32_t ri, uint32_t n) {
  constexpr bool rev = MIRROR && (RHO & ((1 << F) >> 1));
  if constexpr (VEC) {
    *reinterpret_cast<int4*>(keys + (ri & ~3u)) =
        make_int4(x[4 * RHO + (rev ? 3 : 0)], x[4 * RHO + (rev ? 2 : 1)],
                  x[4 * RHO + (rev ? 1 : 2)], x[4 * RHO + (rev ? 0 : 3)]);
  } else {
#pragma unroll
    for (uint32_t c = 0; c < 4; ++c) {
      const uint32_t i = ri ^ c;
      if (i < n) keys[i] = x[4 * RHO + c];
    }
  }
}

// Thread g0 + blockIdx.x * 256 + threadIdx.x.  BOUNDED == false: the
// thread's whole 2^(q+F) block lies below n, every row moves as a 16-byte
// vector and nothing is checked.  Because 256 divides 2^(q-2), a workgroup
// stays inside one block, so a row's address is a workgroup-uniform part
// (block start + row offset, kept in scalar registers) plus one of two
// per-lane 32-bit byte offsets (the column, or its mirror image), which keeps
// the kernel to few vector registers.
// BOUNDED == true: the workgroups of blocks wholly below n run as above; in
// the block that straddles n rows wholly below n move as vectors, a row that
// straddles n goes key by key, rows at or past n are sentinels -- one launch
// for any n.
// A pass is never the first or last kernel of a sort, so keys are in the
// sorting domain on both sides and no codec is applied.
template <int F, bool MIRROR, bool BOUNDED>
__global__ __launch_bounds__(256) void global_pass_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                          int q, uint32_t g0) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  bool whole = true;  // uniform: the workgroup's block lies wholly below n
  if constexpr (BOUNDED)
    whole = ((uint64_t)(((g0 + blockIdx.x * 256u) >> (q - 2)) + 1u) << (q + F)) <= (uint64_t)n;
  // each path has its own key array: the checked path's may live in
  // scratch memory, which must not pull the unchecked path's there too
  if (whole) {
    int32_t x[4 * ROWS];
    const uint32_t gw = g0 + blockIdx.x * 256u;            // uniform
    const uint32_t blk = gw >> (q - 2);                    // uniform block index
    int32_t* bp = keys + ((size_t)blk << (q + F));         // uniform block start
    const uint32_t col = ((gw + threadIdx.x) & ((1u << (q - 2)) - 1u)) << 2;
    const uint32_t off = col * 4u;                          // byte offset, < 2^(q+2)
    const uint32_t moff = ((1u << q) - 4u - col) * 4u;      // mirrored column
    auto row_ptr = [&](int rho) -> int4* {
      const bool mir = MIRROR && (rho & TOP);
      const uint32_t r = mir ? ((uint32_t)(ROWS - 1) ^ (uint32_t)(rho & (TOP - 1))) : (uint32_t)rho;
      char* rb = reinterpret_cast<char*>(bp + ((size_t)r << q));
      return reinterpret_cast<int4*>(rb + (mir ? moff : off));
    };
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool rev = MIRROR && (RHO & TOP);
      const int4 v = *row_ptr(RHO);
      x[4 * RHO + (rev ? 3 : 0)] = v.x;
      x[4 * RHO + (rev ? 2 : 1)] = v.y;
      x[4 * RHO + (rev ? 1 : 2)] = v.z;
      x[4 * RHO + (rev ? 0 : 3)] = v.w;
    });
    // Scheduling fences keep the compiler from interleaving the steps with
    // the loads and stores, which would hold many more registers live.
    __builtin_amdgcn_sched_barrier(0);
    pass_steps<F, MIRROR>(x);
    __builtin_amdgcn_sched_barrier(0);
    static_for<0, ROWS>([&](auto RHO) {
      constexpr bool rev = MIRROR && (RHO & TOP);
      *row_ptr(RHO) = make_int4(x[4 * RHO + (rev ? 3 : 0)], x[4 * RHO + (rev ? 2 : 1)],
                                x[4 * RHO + (rev ? 1 : 2)], x[4 * RHO + (rev ? 0 : 3)]);
      __builtin_amdgcn_sched_barrier(0);
    });
  } else if constexpr (BOUNDED) {
    int32_t x[4 * ROWS];
    const uint32_t g = g0 + blockIdx.x * 256u + threadIdx.x;
    const uint32_t lowmask = (1u << (q - 2)) - 1u;
    const uint32_t base = ((g & lowmask) << 2) | ((g >> (q - 2)) << (q + F));
    if (base >= n) return;
    const uint32_t span = (q + F >= 32) ? 0xFFFFFFFFu : ((1u << (q + F)) - 1u);
    static_for<0, ROWS>([&](auto RHO) {
      const uint32_t ri = pass_row_index<F, MIRROR, RHO>(base, span, q);
      if ((ri | 3u) < n)
        pass_load_row<F, MIRROR, RHO, true>(x, keys, ri, n);
      else
        pass_load_row<F, MIRROR, RHO, false>(x, keys, ri, n);
    });
    pass_steps<F, MIRROR>(x);
    static_for<0, ROWS>([&](auto RHO) {
      const uint32_t ri = pass_row_index<F, MIRROR, RHO>(base, span, q);
      if ((ri | 3u) < n)
        pass_store_row<F, MIRROR, RHO, true>(x, keys, ri, n);
      else
        pass_store_row<F, MIRROR, RHO, false>(x, keys, ri, n);
    });
  }
}

// ---------------------------------------------------------------------------
// launchers

// Thread counts of a pass (see global_pass_kernel's mapping): `full` threads
// own keys in 2^(q+f) blocks wholly below n, `total` own any key below n.
static void global_pass_threads(uint32_t n, int q, int f, uint32_t* full, uint32_t* total) {
  const uint64_t per_block = 1ull << (q - 2);
  const uint64_t nfull = (uint64_t)n >> (q + f);
  const uint64_t rem = (uint64_t)n & ((1ull << (q + f)) - 1);
  uint64_t part = (rem + 3) >> 2;
  if (part > per_block) part = per_block;
  *full = (uint32_t)(nfull * per_block);
  *total = (uint32_t)(nfull * per_block + part);
}

template <int F, bool MIRROR>
static void launch_global_FM(int32_t* keys, uint32_t n, int q, hipStream_t st) {
  uint32_t full = 0, total = 0;
  global_pass_threads(n, q, F, &full, &total);
  if (total == full)  // full is a multiple of 2^(q-2) >= 256
    global_pass_kernel<F, MIRROR, false><<<full / 256, 256, 0, st>>>(keys, n, q, 0u);
  else  // one launch: whole blocks unchecked, the straddling block checked
    global_pass_kernel<F, MIRROR, true><<<(total + 255) / 256, 256, 0, st>>>(keys, n, q, 0u);
}

template <int F>
static void launch_global_F(bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  if (mirror)
    launch_global_FM<F, true>(keys, n, q, st);
  else
    launch_global_FM<F, false>(keys, n, q, st);
}

void launch_global_pass(int f, bool mirror, int32_t* keys, uint32_t n, int q, hipStream_t st) {
  switch (f) {
    case 1: launch_global_F<1>(mirror, keys, n, q, st); break;
    case 2: launch_global_F<2>(mirror, keys, n, q, st); break;
    case 3: launch_global_F<3>(mirror, keys, n, q, st); break;
    case 4: launch_global_F<4>(mirror, keys, n, q, st); break;
    case 5: launch_global_F<5>(mirror, keys, n, q, st); break;
    // wider fusion: one column of 2^f keys per thread (kernels_column.hip)
    default: launch_column_pass_i32(f, mirror, keys, n, q, st); break;
  }
}

}  // namespace bitonic
