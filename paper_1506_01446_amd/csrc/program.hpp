// Compile-time description of how a tile of 2^L keys moves through registers.
//
// A workgroup of 2^(L-r) threads holds a tile of 2^L keys, R = 2^r keys per
// thread.  Which keys a thread holds is given by a "layout": r basis vectors
// v[0..r) over GF(2) (tile indices read as bit vectors).  Thread t holds the
// keys at indices  base(t) XOR off(j)  for register slots j in [0, R), where
// off(j) is the XOR of the v[m] whose bit m is set in j and base(t) spreads
// the bits of t over the index bits that are not the leading bit of any
// v[m].  A basis vector is either a single index bit 2^b or the mirror
// vector 2^p - 1, which pairs a key with its mirror image inside its 2^p
// block (the first step of phase p in the flip arrangement of the network).
//
// A compare-exchange step is a register mask D: slot j meets slot j XOR D,
// and the key that sits at the lower tile index takes the minimum.  Which
// slot that is only depends on j and the layout (the leading bit of
// off(D) is zero in base(t)), so it is decided at compile time and the step
// compiles to straight v_min_i32 / v_max_i32 pairs.
//
// A program is a list of groups (layout + steps).  Keys are loaded from
// global memory in the first group's layout, move between groups through
// LDS, and are stored from the last group's layout.
#pragma once

#include <stdint.h>

namespace bitonic {

constexpr int kMaxRegBits = 6;
constexpr int kMaxSteps = 28;
constexpr int kMaxGroups = 40;

struct Group {
  int r = 0;
  uint32_t v[kMaxRegBits] = {};
  int nsteps = 0;
  uint32_t d[kMaxSteps] = {};
};

struct Program {
  int L = 0;
  int r = 0;
  int ngroups = 0;
  Group g[kMaxGroups] = {};
};

constexpr int highbit(uint32_t x) {
  int h = -1;
  while (x) {
    ++h;
    x >>= 1;
  }
  return h;
}

// Offset of register slot j inside the thread's key set.
constexpr uint32_t goff(const Group& G, uint32_t j) {
  uint32_t o = 0;
  for (int m = 0; m < G.r; ++m)
    if ((j >> m) & 1u) o ^= G.v[m];
  return o;
}

// Index bits that carry the thread id: all tile bits except leading bits.
constexpr uint32_t free_mask(const Group& G, int L) {
  uint32_t lead = 0;
  for (int m = 0; m < G.r; ++m) lead |= 1u << highbit(G.v[m]);
  return ((L >= 32) ? 0xFFFFFFFFu : ((1u << L) - 1u)) & ~lead;
}

// True if slot j holds the lower tile index of the pair (j, j ^ D).
constexpr bool slot_is_lower(const Group& G, uint32_t j, uint32_t D) {
  const int h = highbit(goff(G, D));
  return ((goff(G, j) >> h) & 1u) == 0;
}

// Layout for global loads and stores: each thread holds 4 consecutive keys
// (index bits 0, 1) of r - 2 rows (the top tile bits), so a wave moves 64
// consecutive 16-byte pieces per instruction.
constexpr Group io_group(int L, int r) {
  Group G{};
  G.r = r;
  G.v[0] = 1u;
  G.v[1] = 2u;
  for (int m = 2; m < r; ++m) G.v[m] = 1u << (L - 1 - (m - 2));
  return G;
}

// Layout for scalar global loads and stores (keys not 16-byte aligned, e.g.
// segments): the registers hold the top r tile bits, so lanes step through
// consecutive keys.
constexpr Group io_scalar_group(int L, int r) {
  Group G{};
  G.r = r;
  for (int m = 0; m < r; ++m) G.v[m] = 1u << (L - 1 - m);
  return G;
}

constexpr Group blocked_group(int r) {
  Group G{};
  G.r = r;
  for (int m = 0; m < r; ++m) G.v[m] = 1u << m;
  return G;
}

// Bits top..0 of one merge, in groups of r bits from the top.  If `mirror`,
// the first step is the phase's mirror step (bit top pairs mirror images).
constexpr void add_merge_bits(Program& P, int top, bool mirror) {
  const int r = P.r;
  while (top >= r) {
    Group G{};
    G.r = r;
    for (int m = 0; m < r; ++m) G.v[m] = 1u << (top - m);
    if (mirror) G.v[0] = (2u << top) - 1u;
    for (int m = 0; m < r; ++m) G.d[G.nsteps++] = 1u << m;
    mirror = false;
    P.g[P.ngroups++] = G;
    top -= r;
  }
  if (top >= 0) {
    Group G = blocked_group(r);
    if (mirror) {
      G.d[G.nsteps++] = (2u << top) - 1u;
      --top;
    }
    for (int b = top; b >= 0; --b) G.d[G.nsteps++] = 1u << b;
    P.g[P.ngroups++] = G;
  }
}

// Phases 1..L of the flip network on one tile: afterwards the tile is
// ascending.  Phases 1..r run in the blocked layout (thread holds R
// consecutive keys).
constexpr Program make_tile_sort(int L, int r) {
  Program P{};
  P.L = L;
  P.r = r;
  P.g[P.ngroups++] = io_group(L, r);
  Group g0 = blocked_group(r);
  const int pin = L < r ? L : r;
  for (int p = 1; p <= pin; ++p) {
    g0.d[g0.nsteps++] = (1u << p) - 1u;          // mirror step of phase p
    for (int b = p - 2; b >= 0; --b) g0.d[g0.nsteps++] = 1u << b;
  }
  P.g[P.ngroups++] = g0;
  for (int p = r + 1; p <= L; ++p) add_merge_bits(P, p - 1, true);
  P.g[P.ngroups++] = io_group(L, r);
  return P;
}

// The last L steps of a phase longer than the tile: strides 2^(L-1) .. 1,
// smaller key to the lower index, on each tile.  The first layout also holds
// index bits 0 and 1, so every thread loads 4 consecutive keys at a time.
constexpr Program make_tile_merge(int L, int r) {
  Program P{};
  P.L = L;
  P.r = r;
  Group G{};
  G.r = r;
  G.v[0] = 1u;
  G.v[1] = 2u;
  for (int m = 2; m < r; ++m) {
    G.v[m] = 1u << (L - 1 - (m - 2));
    G.d[G.nsteps++] = 1u << m;
  }
  P.g[P.ngroups++] = G;
  add_merge_bits(P, L - 1 - (r - 2), false);
  P.g[P.ngroups++] = io_group(L, r);
  return P;
}

// Phases 1..L with scalar I/O.  A tile of L == r bits is one thread's
// registers: a single blocked group and no LDS.
constexpr Program make_tile_sort_scalar(int L, int r) {
  Program P{};
  P.L = L;
  P.r = r;
  if (L > r) P.g[P.ngroups++] = io_scalar_group(L, r);
  Group g0 = blocked_group(r);
  const int pin = L < r ? L : r;
  for (int p = 1; p <= pin; ++p) {
    g0.d[g0.nsteps++] = (1u << p) - 1u;
    for (int b = p - 2; b >= 0; --b) g0.d[g0.nsteps++] = 1u << b;
  }
  P.g[P.ngroups++] = g0;
  for (int p = r + 1; p <= L; ++p) add_merge_bits(P, p - 1, true);
  if (L > r) P.g[P.ngroups++] = io_scalar_group(L, r);
  return P;
}

// Strides 2^(L-1) .. 1 with scalar I/O: the first merge group's layout (the
// top r bits in registers) is already the scalar I/O layout.
constexpr Program make_tile_merge_scalar(int L, int r) {
  Program P{};
  P.L = L;
  P.r = r;
  add_merge_bits(P, L - 1, false);
  P.g[P.ngroups++] = io_scalar_group(L, r);
  return P;
}

// Program kinds: 0 sort, 1 merge (16-byte vector I/O); 2 sort, 3 merge
// (scalar I/O).
constexpr Program make_program(int L, int r, int kind) {
  return kind == 0   ? make_tile_sort(L, r)
         : kind == 1 ? make_tile_merge(L, r)
         : kind == 2 ? make_tile_sort_scalar(L, r)
                     : make_tile_merge_scalar(L, r);
}

constexpr bool layout_is_vector4(const Group& G) {
  return G.r >= 2 && G.v[0] == 1u && G.v[1] == 2u;
}

// Every basis vector a single index bit: then base(t) and off(j) have no bit
// in common and base ^ off == base + off.
constexpr bool layout_is_unit(const Group& G) {
  for (int m = 0; m < G.r; ++m)
    if ((G.v[m] & (G.v[m] - 1u)) != 0) return false;
  return true;
}

// The LDS swizzle of device.hpp, which is linear over XOR.
constexpr uint32_t swz_const(uint32_t i) { return i ^ ((i >> 5) & 31u); }

// Total compare-exchange steps a program performs (for checks).
constexpr int program_steps(const Program& P) {
  int s = 0;
  for (int g = 0; g < P.ngroups; ++g) s += P.g[g].nsteps;
  return s;
}

}  // namespace bitonic
