// Kernels of the single-array sort.
//
//  tile_kernel<L, r, 0>   phases 1..L of the network on every 2^L tile, keys
//                         in registers, regrouped through LDS (the paper's
//                         shared-memory optimization, section 4.1, with the
//                         register blocking of section 4.2 inside the tile)
//  tile_kernel<L, r, 1>   the last L steps (strides 2^(L-1)..1) of a phase
//                         longer than the tile, on every tile
//  global_pass_kernel<F>  F consecutive steps with strides >= 2^q in one pass
//                         over HBM: each thread holds 4 columns x 2^F rows of
//                         keys in registers (section 4.2, generalised from
//                         2 steps to F); for F = 6, 7 the one-column kernel of
//                         column_pass.hpp
//  lds_network_kernel     the same network steps with one compare-exchange per
//                         thread per step in LDS (section 4.1 as written)
//  step_kernel            one step, one compare-exchange per thread, in global
//                         memory (the basic scheme of section 3.3)
//
// All kernels sort ascending in the codec domain (see Codec) and treat indices
// >= n as absent INT32_MAX sentinels.  The tile and pass kernels of a sort
// apply the codec only where the sort's data enters and leaves them (CX, see
// KeyIO); the LDS-network and step kernels apply it at every access.
#include "column_pass.hpp"
#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

// One tile per workgroup.
template <int L, int RL, int KIND, int CX>
__global__ __launch_bounds__(1 << (L - RL)) void tile_kernel(int32_t* __restrict__ keys,
                                                             uint32_t n, Codec codec) {
  using PR = Prog<L, RL, KIND>;
  __shared__ int32_t lds[PR::LDSW];
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < (uint32_t)PR::T ? left : (uint32_t)PR::T;
  tile_program<PR>(keys + t0, valid, KeyIO<CX>{codec}, lds, threadIdx.x);
}

// The full tiles blockIdx.x, blockIdx.x + gridDim.x, ... of keys[0, n), then
// the partial last tile (if any) on one block.  The keys of a block's next
// tile are loaded into a second register set before the current tile's steps
// run, so that those loads are in flight while the tile is processed and
// stored (the workgroup barriers wait for LDS traffic only).  The next tile is
// read through a buffer resource that is empty when there is no next tile, so
// every iteration issues the same loads: with a load in a branch the
// compiler would wait for all loads at the join, the prefetch included.  The
// thread id is passed through an empty asm statement every iteration so that
// the compiler recomputes the loop-invariant LDS and global offsets instead
// of keeping all of them live in registers.
template <int L, int RL, int KIND, int CX>
__global__ __launch_bounds__(1 << (L - RL)) void tile_loop_kernel(int32_t* __restrict__ keys,
                                                                  uint32_t n, Codec codec) {
  using PR = Prog<L, RL, KIND>;
  constexpr int LAST = PR::value.ngroups - 1;
  static_assert(layout_is_vector4(PR::value.g[LAST]), "16-byte store layout expected");
  const KeyIO<CX> cd{codec};
  __shared__ int32_t lds[PR::LDSW];
  const uint32_t nfull = n >> L;
  auto rsrc_of = [&](uint32_t tile) {
    return tile_rsrc(keys + ((size_t)tile << L), tile < nfull ? (uint32_t)PR::T * 4u : 0u);
  };
  uint32_t tile = blockIdx.x;
  int32_t x[PR::R];
  load_tile_rsrc<PR, 0>(x, rsrc_of(tile), cd, threadIdx.x);
  // Wait for the first tile here, so that at the loop head only the
  // previous iteration's prefetch has to be waited for, not its stores.
#pragma unroll
  for (int j = 0; j < PR::R; ++j) asm volatile("" : "+v"(x[j]));
  for (; tile < nfull; tile += gridDim.x) {
    uint32_t tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    int32_t y[PR::R];
    load_tile_rsrc<PR, 0>(y, rsrc_of(tile + gridDim.x), cd, tid);
    run_from<PR, 0>(x, lds, tid);
    store_tile<PR, LAST>(x, keys + ((size_t)tile << L), (uint32_t)PR::T, cd, tid);
    static_for<0, PR::R>([&](auto J) { x[J] = y[J]; });
  }
  const uint32_t rest = n & (uint32_t)(PR::T - 1);
  if (rest != 0 && blockIdx.x == nfull % gridDim.x)
    tile_program<PR>(keys + ((size_t)nfull << L), rest, cd, lds, threadIdx.x);
}

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
// BOUNDED == true: rows wholly below n move as vectors, a row that straddles
// n goes key by key, rows at or past n are sentinels.
// A pass is never the first or last kernel of a sort, so keys are in the
// sorting domain on both sides and no codec is applied.
template <int F, bool MIRROR, bool BOUNDED>
__global__ __launch_bounds__(256) void global_pass_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                          int q, uint32_t g0) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  int32_t x[4 * ROWS];
  if constexpr (!BOUNDED) {
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
  } else {
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

// One step in LDS per iteration: comparator c of the step (lower index i has
// bit sb clear) meets i | 2^sb, or its mirror i ^ (2^(sb+1) - 1).
__device__ __forceinline__ void lds_step(int32_t* s, uint32_t T, int sb, bool mirror) {
  for (uint32_t c = threadIdx.x; c < (T >> 1); c += blockDim.x) {
    const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
    const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
    const int32_t a = s[i], b = s[j];
    s[i] = min(a, b);
    s[j] = max(a, b);
  }
  __syncthreads();
}

// Tile of 2^L keys (L <= 13) in LDS.  tail == 0: phases p_first..p_last
// (each a mirror step and half-cleaners); tail != 0: strides 2^(L-1)..1.
__global__ __launch_bounds__(1024) void lds_network_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                           int L, int p_first, int p_last,
                                                           int tail, Codec cd) {
  extern __shared__ int32_t s[];
  const uint32_t T = 1u << L;
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < T ? left : T;
  for (uint32_t i = threadIdx.x; i < T; i += blockDim.x)
    s[i] = i < valid ? cd.enc(keys[t0 + i]) : kPad;
  __syncthreads();
  if (tail) {
    for (int sb = L - 1; sb >= 0; --sb) lds_step(s, T, sb, false);
  } else {
    for (int p = p_first; p <= p_last; ++p) {
      lds_step(s, T, p - 1, true);
      for (int sb = p - 2; sb >= 0; --sb) lds_step(s, T, sb, false);
    }
  }
  for (uint32_t i = threadIdx.x; i < valid; i += blockDim.x) keys[t0 + i] = cd.dec(s[i]);
}

// One step of the network in global memory, one comparator per thread.
__global__ __launch_bounds__(256) void step_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                   uint32_t half, int sb, int mirror,
                                                   Codec cd) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= half) return;
  const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
  const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
  if (j >= n) return;
  const int32_t a = cd.enc(keys[i]), b = cd.enc(keys[j]);
  if (a > b) {
    keys[i] = cd.dec(b);
    keys[j] = cd.dec(a);
  }
}

// ---------------------------------------------------------------------------
// launchers

constexpr int kTileRegLog = kTileRegLogPlain;

template <int L, int CX>
static void launch_merge_LC(int32_t* keys, uint32_t n, Codec cd, uint32_t max_blocks,
                            hipStream_t st) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (max_blocks == 0 || max_blocks >= ntiles)
    tile_kernel<L, kTileRegLog, 1, CX><<<ntiles, NT, 0, st>>>(keys, n, cd);
  else
    tile_loop_kernel<L, kTileRegLog, 1, CX><<<max_blocks, NT, 0, st>>>(keys, n, cd);
}

// Instantiated codec modes: a tile sort is a sort's first kernel (CX_ENC, or
// CX_BOTH when it is the only one), a merge is never its first (CX_DEC for the
// last); CX_NONE serves the identity codec and the kernels in between.
template <int L>
static void launch_tile_L(int kind, int32_t* keys, uint32_t n, Codec cd, int cx,
                          uint32_t max_blocks, hipStream_t st) {
  const uint32_t ntiles = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (codec_is_identity(cd)) cx = CX_NONE;
  if (kind == 0) {
    if (cx == CX_NONE)
      tile_kernel<L, kTileRegLog, 0, CX_NONE><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else if (cx == CX_ENC)
      tile_kernel<L, kTileRegLog, 0, CX_ENC><<<ntiles, NT, 0, st>>>(keys, n, cd);
    else
      tile_kernel<L, kTileRegLog, 0, CX_BOTH><<<ntiles, NT, 0, st>>>(keys, n, cd);
  } else if (cx == CX_NONE) {
    launch_merge_LC<L, CX_NONE>(keys, n, cd, max_blocks, st);
  } else {
    launch_merge_LC<L, CX_DEC>(keys, n, cd, max_blocks, st);
  }
}

bool tile_log2_supported(int L) { return L >= kTileMinLog2 && L <= kTileMaxLog2; }

void launch_tile(int L, int kind, int32_t* keys, uint32_t n, Codec cd, int cx,
                 uint32_t max_blocks, hipStream_t st) {
  switch (L) {
    case 11: launch_tile_L<11>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 12: launch_tile_L<12>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 13: launch_tile_L<13>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 14: launch_tile_L<14>(kind, keys, n, cd, cx, max_blocks, st); break;
    case 15: launch_tile_L<15>(kind, keys, n, cd, cx, max_blocks, st); break;
    default: break;
  }
}

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
  if (full > 0)  // full is a multiple of 2^(q-2) >= 256
    global_pass_kernel<F, MIRROR, false><<<full / 256, 256, 0, st>>>(keys, n, q, 0u);
  if (total > full)
    global_pass_kernel<F, MIRROR, true><<<(total - full + 255) / 256, 256, 0, st>>>(keys, n, q,
                                                                                  full);
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
    // wider fusion: one column of 2^f keys per thread (the same 128 keys at
    // f = 7 as four columns at f = 5), 256 B per wave access
    case 6: launch_column_pass_F<6>(mirror, Keys32{keys}, n, q, st); break;
    case 7: launch_column_pass_F<7>(mirror, Keys32{keys}, n, q, st); break;
    default: break;
  }
}

void launch_lds_network(int L, int p_first, int p_last, bool tail, int32_t* keys, uint32_t n,
                        Codec cd, hipStream_t st) {
  const uint32_t T = 1u << L;
  const uint32_t blocks = (uint32_t)(((uint64_t)n + T - 1) >> L);
  uint32_t threads = T / 2;
  if (threads > 1024) threads = 1024;
  if (threads < 64) threads = 64;
  lds_network_kernel<<<blocks, threads, T * sizeof(int32_t), st>>>(keys, n, L, p_first, p_last,
                                                                   tail ? 1 : 0, cd);
}

void launch_step(int sb, bool mirror, int32_t* keys, uint32_t n, uint32_t N, Codec cd,
                 hipStream_t st) {
  const uint32_t half = N >> 1;
  const uint32_t blocks = (half + 255) / 256;
  step_kernel<<<blocks, 256, 0, st>>>(keys, n, half, sb, mirror ? 1 : 0, cd);
}

}  // namespace bitonic
