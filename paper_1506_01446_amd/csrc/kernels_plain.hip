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
//                         2 steps to F)
//  lds_network_kernel     the same network steps with one compare-exchange per
//                         thread per step in LDS (section 4.1 as written)
//  step_kernel            one step, one compare-exchange per thread, in global
//                         memory (the basic scheme of section 3.3)
//
// All kernels sort ascending in the XOR domain (key ^ flip) and treat indices
// >= n as absent INT32_MAX sentinels.
#include "device.hpp"
#include "launch.hpp"

namespace bitonic {

template <int L, int RL, int KIND>
__global__ __launch_bounds__(1 << (L - RL)) void tile_kernel(int32_t* __restrict__ keys,
                                                             uint32_t n, int32_t flip) {
  using PR = Prog<L, RL, KIND>;
  __shared__ int32_t lds[PR::T];
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < (uint32_t)PR::T ? left : (uint32_t)PR::T;
  tile_program<PR>(keys + t0, valid, flip, lds, threadIdx.x);
}

// Keys of thread g: 4 consecutive columns x 2^F rows.  Row rho sits at
// index base | rho << q; with MIRROR the upper half of the rows are the
// mirror images (index XOR (2^(q+F) - 1)), so the first step pairs each key
// with its mirror in the 2^(q+F) block.
template <int F, bool MIRROR>
__global__ __launch_bounds__(256) void global_pass_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                          int q, int32_t flip) {
  constexpr int ROWS = 1 << F;
  constexpr int TOP = ROWS >> 1;
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  const uint32_t lowmask = (1u << (q - 2)) - 1u;
  const uint32_t base = ((g & lowmask) << 2) | ((g >> (q - 2)) << (q + F));
  if (base >= n) return;
  const uint32_t span = (q + F >= 32) ? 0xFFFFFFFFu : ((1u << (q + F)) - 1u);

  int32_t x[4 * ROWS];
  auto row_index = [&](int rho) -> uint32_t {
    if (MIRROR && (rho & TOP)) return base ^ span ^ ((uint32_t)(rho & (TOP - 1)) << q);
    return base | ((uint32_t)rho << q);
  };
  const bool inside = (base | span) < n;

  if (inside) {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      constexpr bool rev = MIRROR && (rho & TOP);
      const uint32_t ri = row_index(rho);
      const int4 v = *reinterpret_cast<const int4*>(keys + (ri & ~3u));
      if constexpr (rev) {
        x[4 * rho + 0] = v.w ^ flip;
        x[4 * rho + 1] = v.z ^ flip;
        x[4 * rho + 2] = v.y ^ flip;
        x[4 * rho + 3] = v.x ^ flip;
      } else {
        x[4 * rho + 0] = v.x ^ flip;
        x[4 * rho + 1] = v.y ^ flip;
        x[4 * rho + 2] = v.z ^ flip;
        x[4 * rho + 3] = v.w ^ flip;
      }
    });
  } else {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      const uint32_t ri = row_index(rho);
      static_for<0, 4>([&](auto C) {
        const uint32_t i = ri ^ (uint32_t)C;
        x[4 * rho + C] = i < n ? (keys[i] ^ flip) : kPad;
      });
    });
  }

  if constexpr (MIRROR) {
    static_for<0, TOP>([&](auto RHO) {
      static_for<0, 4>([&](auto C) { cmpx(x[4 * RHO + C], x[4 * (RHO + TOP) + C]); });
    });
  }
  constexpr int NB = MIRROR ? F - 1 : F;  // remaining row bits, highest first
  static_for<0, NB>([&](auto I) {
    constexpr int b = NB - 1 - I;
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      constexpr int partner = rho ^ (1 << b);
      if constexpr (rho < partner) {
        // rho has bit b clear; in a mirrored upper half the order is reversed
        constexpr bool low = !(MIRROR && (rho & TOP));
        static_for<0, 4>([&](auto C) {
          if constexpr (low) {
            cmpx(x[4 * rho + C], x[4 * partner + C]);
          } else {
            cmpx(x[4 * partner + C], x[4 * rho + C]);
          }
        });
      }
    });
  });

  if (inside) {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      constexpr bool rev = MIRROR && (rho & TOP);
      const uint32_t ri = row_index(rho);
      int4 v;
      if constexpr (rev) {
        v = make_int4(x[4 * rho + 3] ^ flip, x[4 * rho + 2] ^ flip, x[4 * rho + 1] ^ flip,
                      x[4 * rho + 0] ^ flip);
      } else {
        v = make_int4(x[4 * rho + 0] ^ flip, x[4 * rho + 1] ^ flip, x[4 * rho + 2] ^ flip,
                      x[4 * rho + 3] ^ flip);
      }
      *reinterpret_cast<int4*>(keys + (ri & ~3u)) = v;
    });
  } else {
    static_for<0, ROWS>([&](auto RHO) {
      constexpr int rho = RHO;
      const uint32_t ri = row_index(rho);
      static_for<0, 4>([&](auto C) {
        const uint32_t i = ri ^ (uint32_t)C;
        if (i < n) keys[i] = x[4 * rho + C] ^ flip;
      });
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
                                                           int tail, int32_t flip) {
  extern __shared__ int32_t s[];
  const uint32_t T = 1u << L;
  const uint32_t t0 = (uint32_t)blockIdx.x << L;
  const uint32_t left = n - t0;
  const uint32_t valid = left < T ? left : T;
  for (uint32_t i = threadIdx.x; i < T; i += blockDim.x)
    s[i] = i < valid ? (keys[t0 + i] ^ flip) : kPad;
  __syncthreads();
  if (tail) {
    for (int sb = L - 1; sb >= 0; --sb) lds_step(s, T, sb, false);
  } else {
    for (int p = p_first; p <= p_last; ++p) {
      lds_step(s, T, p - 1, true);
      for (int sb = p - 2; sb >= 0; --sb) lds_step(s, T, sb, false);
    }
  }
  for (uint32_t i = threadIdx.x; i < valid; i += blockDim.x) keys[t0 + i] = s[i] ^ flip;
}

// One step of the network in global memory, one comparator per thread.
__global__ __launch_bounds__(256) void step_kernel(int32_t* __restrict__ keys, uint32_t n,
                                                   uint32_t half, int sb, int mirror,
                                                   int32_t flip) {
  const uint32_t c = blockIdx.x * 256u + threadIdx.x;
  if (c >= half) return;
  const uint32_t i = ((c >> sb) << (sb + 1)) | (c & ((1u << sb) - 1u));
  const uint32_t j = mirror ? (i ^ ((2u << sb) - 1u)) : (i | (1u << sb));
  if (j >= n) return;
  const int32_t a = keys[i] ^ flip, b = keys[j] ^ flip;
  if (a > b) {
    keys[i] = b ^ flip;
    keys[j] = a ^ flip;
  }
}

// ---------------------------------------------------------------------------
// launchers

constexpr int kTileRegLog = 5;  // 32 keys per thread in the tile kernels

template <int L>
static void launch_tile_L(int kind, int32_t* keys, uint32_t n, int32_t flip, hipStream_t st) {
  const uint32_t blocks = (uint32_t)(((uint64_t)n + (1u << L) - 1) >> L);
  constexpr int NT = 1 << (L - kTileRegLog);
  if (kind == 0)
    tile_kernel<L, kTileRegLog, 0><<<blocks, NT, 0, st>>>(keys, n, flip);
  else
    tile_kernel<L, kTileRegLog, 1><<<blocks, NT, 0, st>>>(keys, n, flip);
}

bool tile_log2_supported(int L) { return L >= kTileMinLog2 && L <= kTileMaxLog2; }

void launch_tile(int L, int kind, int32_t* keys, uint32_t n, int32_t flip, hipStream_t st) {
  switch (L) {
    case 11: launch_tile_L<11>(kind, keys, n, flip, st); break;
    case 12: launch_tile_L<12>(kind, keys, n, flip, st); break;
    case 13: launch_tile_L<13>(kind, keys, n, flip, st); break;
    default: break;
  }
}

// Threads whose base index is below n (see global_pass_kernel's mapping).
static uint32_t global_pass_threads(uint32_t n, int q, int f) {
  const uint64_t per_block = 1ull << (q - 2);
  const uint64_t full = (uint64_t)n >> (q + f);
  const uint64_t rem = (uint64_t)n & ((1ull << (q + f)) - 1);
  uint64_t part = (rem + 3) >> 2;
  if (part > per_block) part = per_block;
  return (uint32_t)(full * per_block + part);
}

template <int F>
static void launch_global_F(bool mirror, int32_t* keys, uint32_t n, int q, int32_t flip,
                            hipStream_t st) {
  const uint32_t threads = global_pass_threads(n, q, F);
  const uint32_t blocks = (threads + 255) / 256;
  if (blocks == 0) return;
  if (mirror)
    global_pass_kernel<F, true><<<blocks, 256, 0, st>>>(keys, n, q, flip);
  else
    global_pass_kernel<F, false><<<blocks, 256, 0, st>>>(keys, n, q, flip);
}

void launch_global_pass(int f, bool mirror, int32_t* keys, uint32_t n, int q, int32_t flip,
                        hipStream_t st) {
  switch (f) {
    case 1: launch_global_F<1>(mirror, keys, n, q, flip, st); break;
    case 2: launch_global_F<2>(mirror, keys, n, q, flip, st); break;
    case 3: launch_global_F<3>(mirror, keys, n, q, flip, st); break;
    case 4: launch_global_F<4>(mirror, keys, n, q, flip, st); break;
    case 5: launch_global_F<5>(mirror, keys, n, q, flip, st); break;
    default: break;
  }
}

void launch_lds_network(int L, int p_first, int p_last, bool tail, int32_t* keys, uint32_t n,
                        int32_t flip, hipStream_t st) {
  const uint32_t T = 1u << L;
  const uint32_t blocks = (uint32_t)(((uint64_t)n + T - 1) >> L);
  uint32_t threads = T / 2;
  if (threads > 1024) threads = 1024;
  if (threads < 64) threads = 64;
  lds_network_kernel<<<blocks, threads, T * sizeof(int32_t), st>>>(keys, n, L, p_first, p_last,
                                                                   tail ? 1 : 0, flip);
}

void launch_step(int sb, bool mirror, int32_t* keys, uint32_t n, uint32_t N, int32_t flip,
                 hipStream_t st) {
  const uint32_t half = N >> 1;
  const uint32_t blocks = (half + 255) / 256;
  step_kernel<<<blocks, 256, 0, st>>>(keys, n, half, sb, mirror ? 1 : 0, flip);
}

}  // namespace bitonic
