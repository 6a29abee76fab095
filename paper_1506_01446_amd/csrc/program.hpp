// Compile-time description of how a tile of 2^L keys moves through registers.
//
// A workgroup of 2^(L-r) threads holds a tile of 2^L keys, R = 2^r keys per
// thread.  Which keys a thread holds is given by a "layout": r distinct index
// bits b[0..r) (the basis vectors v[m] = 2^b[m]).  Thread t holds register
// slots j in [0, R); slot j sits at tile index base(t) + off(j), where off(j)
// is the sum of the v[m] whose bit m is set in j and base(t) spreads the bits
// of t over the index bits that are not basis bits.  base and off share no
// bit, so base + off == base | off.
//
// The first step of phase p compares each key with its mirror image inside
// its 2^p block (index i XOR (2^p - 1)).  A layout that starts phase p is
// "virtual": its keys are read so that the upper half of every 2^p block is
// mirrored -- virtual index v holds the key of real index m(v), where
// m(v) = v XOR (2^(p-1) - 1) if bit p-1 of v is set and m(v) = v otherwise
// (m is its own inverse).  In virtual indices the mirror step pairs v with
// v XOR 2^(p-1), a single bit, and the later steps of the phase keep their
// strides but run in the opposite direction in the mirrored half.
//
// A compare-exchange step is a register mask D: slot j meets slot j XOR D, and
// the key at the lower real index takes the minimum.  Which slot that is only
// depends on j and the layout, so it is decided at compile time and the step
// compiles to straight v_min_i32 / v_max_i32 pairs.
//
// A "lane step" (a nonzero lane part, D >> 8) pairs slot j of lane l with
// slot j XOR (D & 0xFF) of lane l XOR (D >> 8) of the same wave: a step on
// index bits that the layout maps to lane bits, done with cross-lane moves
// (DPP) instead of a regroup through LDS.  Lane steps occur only in the
// blocked layout of the tile sort, where lane bit k is index bit r + k, and
// the highest index bit a lane step flips is always a lane bit, so the lower
// end of each pair is the lane whose bit highbit(D >> 8) is clear.
//
// LDS holds a tile at padded positions P(i) = i + floor(i / 32) (one unused
// word after every 32), which spreads strided accesses over the banks.  P is
// additive over bit-disjoint parts, so the LDS address of a slot is a
// per-thread base P(base) plus a compile-time offset P(off(j)) that fits the
// offset field of the LDS instruction: no address arithmetic per key.
//
// A program is a list of groups (layout + steps).  Keys are loaded from
// global memory in the first group's layout, move between groups through
// LDS, and are stored from the last group's layout.
#pragma once

#include <stdint.h>

namespace bitonic {

constexpr int kMaxRegBits = 6;
constexpr int kMaxSteps = 80;  // a tile of 2^15 keys with lane steps holds 66 in one layout
constexpr int kMaxGroups = 40;

struct Group {
  int r = 0;
  uint32_t v[kMaxRegBits] = {};  // single index bits
  int nsteps = 0;
  uint32_t d[kMaxSteps] = {};
  int vmirror = 0;  // p > 0: virtual indices for phase p (see above)
};

struct Program {
  int L = 0;
  int r = 0;
  int ngroups = 0;
  Group g[kMaxGroups] = {};
};

// The register and lane parts of a step, and a lane step built from them.
constexpr uint32_t step_reg(uint32_t D) { return D & 0xFFu; }
constexpr uint32_t step_lane(uint32_t D) { return D >> 8; }
constexpr uint32_t lane_step(uint32_t lane_mask, uint32_t reg_mask) {
  return (lane_mask << 8) | reg_mask;
}

constexpr int highbit(uint32_t x) {
  int h = -1;
  while (x) {
    ++h;
    x >>= 1;
  }
  return h;
}

// Offset of register slot j inside the thread's key set (virtual index).
constexpr uint32_t goff(const Group& G, uint32_t j) {
  uint32_t o = 0;
  for (int m = 0; m < G.r; ++m)
    if ((j >> m) & 1u) o |= G.v[m];
  return o;
}

constexpr uint32_t reg_mask(const Group& G) {
  uint32_t s = 0;
  for (int m = 0; m < G.r; ++m) s |= G.v[m];
  return s;
}

// Index bits that carry the thread id: all tile bits except basis bits.
constexpr uint32_t free_mask(const Group& G, int L) {
  return ((L >= 32) ? 0xFFFFFFFFu : ((1u << L) - 1u)) & ~reg_mask(G);
}

// Mask applied to the lower bits in the mirrored half of a virtual layout.
constexpr uint32_t mirror_mask(const Group& G) {
  return G.vmirror > 0 ? ((1u << (G.vmirror - 1)) - 1u) : 0u;
}

// Is slot j in the mirrored half (bit p-1 of its virtual index set)?  For a
// virtual layout bit p-1 is always a basis bit, so this is known per slot.
constexpr bool slot_mirrored(const Group& G, uint32_t j) {
  return G.vmirror > 0 && ((goff(G, j) >> (G.vmirror - 1)) & 1u);
}

// Register part of slot j's real index (the thread part is base, or
// base ^ (mirror_mask & free_mask) for mirrored slots).
constexpr uint32_t real_off(const Group& G, uint32_t j) {
  return slot_mirrored(G, j) ? (goff(G, j) ^ (mirror_mask(G) & reg_mask(G))) : goff(G, j);
}

// True if slot j holds the lower real index of the pair (j, j ^ D).
constexpr bool slot_is_lower(const Group& G, uint32_t j, uint32_t D) {
  const int h = highbit(goff(G, D));
  return ((real_off(G, j) >> h) & 1u) == 0;
}

// Padded LDS position of tile index i: one word of padding after every 2^s,
// s = the log2 of the slots per thread.  A regroup's lanes then step through
// LDS in strides that are odd multiples of a word, bank-conflict free for
// the layouts of make_program.  Additive over indices with disjoint bits, so
// a slot's position is P(thread part) + P(register part).
constexpr uint32_t lds_pad(uint32_t i, int s = 5) { return i + (i >> s); }

// Words of LDS a padded tile of 2^L keys occupies.
constexpr uint32_t lds_words(int L, int s = 5) { return lds_pad((1u << L) - 1u, s) + 1u; }

// Index bits that carry a thread's wave number in layout G: the free bits
// left after the lowest six, which carry the lane (64-lane waves; thread t
// is lane t mod 64 of wave t / 64).
constexpr uint32_t wave_bit_mask(const Group& G, int L) {
  uint32_t f = free_mask(G, L);
  for (int k = 0; k < 6 && f; ++k) f &= f - 1;
  return f;
}

// Does a regroup from layout A to layout B keep every key inside the wave
// that holds it?  It does when both layouts put the wave number on the same
// index bits and no mirror of a virtual layout flips one of those bits: the
// set of real indices a wave holds is then the same in A and B.  Such a
// regroup exchanges keys between the lanes of one wave only, so it needs no
// workgroup barrier.  (An exhaustive check over every thread and slot agrees
// with this test on every program the kernels instantiate.)
constexpr bool regroup_in_wave(const Group& A, const Group& B, int L) {
  const uint32_t wa = wave_bit_mask(A, L);
  return wa == wave_bit_mask(B, L) && (wa & mirror_mask(A)) == 0 && (wa & mirror_mask(B)) == 0;
}

// Layout for 16-byte global loads and stores: each thread holds 4
// consecutive keys (index bits 0, 1) of r - 2 rows (the top tile bits), so a
// wave moves 64 consecutive 16-byte pieces per instruction.
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
// the first step is the mirror step of phase top + 1: the first group is a
// virtual layout whose first step pairs bit `top`.
constexpr void add_merge_bits(Program& P, int top, bool mirror) {
  const int r = P.r;
  while (top >= r) {
    Group G{};
    G.r = r;
    for (int m = 0; m < r; ++m) G.v[m] = 1u << (top - m);
    if (mirror) G.vmirror = top + 1;
    for (int m = 0; m < r; ++m) G.d[G.nsteps++] = 1u << m;
    mirror = false;
    P.g[P.ngroups++] = G;
    top -= r;
  }
  if (top >= 0) {
    Group G = blocked_group(r);
    if (mirror) {  // the whole 2^(top+1) block is in registers: mirror pairs
      G.d[G.nsteps++] = (2u << top) - 1u;
      --top;
    }
    for (int b = top; b >= 0; --b) G.d[G.nsteps++] = 1u << b;
    P.g[P.ngroups++] = G;
  }
}

// Phases 1..L of the flip network on one tile: afterwards the tile is
// ascending.  Phases 1..r run in the blocked layout (thread holds R
// consecutive keys, where the mirror step is a register-index mask).  A tile
// of L == r bits is one thread's registers: one group and no LDS.  With
// vector I/O the keys are loaded straight into the blocked layout (R / 4
// 16-byte loads per thread); with scalar I/O they are loaded in the scalar
// I/O layout and regrouped.
//
// lane_top > r (needs a full wave of lanes, L - r >= 6, and L <= 2r + 6):
// steps on index bits that the blocked layout maps to lane bits (bits r ..
// r+5) run there as lane steps where that is cheap.  Phases r+1 .. lane_top
// stay in the blocked layout with no regroup: the mirror step pairs lane l
// with lane l XOR (2^(p-r) - 1) and slot j with slot j XOR (2^r - 1), a
// half-cleaner on bit b pairs lane l with lane l XOR 2^(b-r), and the steps
// on bits below r are register steps.  Phases lane_top+1 .. r+6 regroup
// through LDS as without lane steps.  Longer phases take their top r bits
// (with the mirror step) into the registers of one virtual layout and come
// back to the blocked layout for the rest, its lane bits as lane steps: two
// regroups, both crossing waves, instead of three.  Each lane step costs
// twice the VALU of a register step (a cross-lane move and a v_med3 per
// key), so the choice of lane_top trades VALU for LDS round trips (measured
// on MI355X: lane_top = 9 for 2^14-key tiles).
constexpr void add_lane_merge(int r, Group& blocked, int p, bool in_blocked_mirror) {
  if (in_blocked_mirror) {
    blocked.d[blocked.nsteps++] = lane_step((1u << (p - r)) - 1u, (1u << r) - 1u);
  }
  const int top = in_blocked_mirror ? p - 2 : p - r - 1;
  for (int b = top; b >= r; --b) blocked.d[blocked.nsteps++] = lane_step(1u << (b - r), 0u);
  for (int b = r - 1; b >= 0; --b) blocked.d[blocked.nsteps++] = 1u << b;
}

constexpr Program make_tile_sort(int L, int r, bool vector_io, int lane_top = 0) {
  Program P{};
  P.L = L;
  P.r = r;
  if (L > r && !vector_io) P.g[P.ngroups++] = io_scalar_group(L, r);
  Group g0 = blocked_group(r);
  const int pin = L < r ? L : r;
  for (int p = 1; p <= pin; ++p) {
    g0.d[g0.nsteps++] = (1u << p) - 1u;          // mirror step of phase p
    for (int b = p - 2; b >= 0; --b) g0.d[g0.nsteps++] = 1u << b;
  }
  if (lane_top > r && L - r >= 6 && L <= 2 * r + 6) {
    const int flat = lane_top < L ? (lane_top < r + 6 ? lane_top : r + 6) : L;
    for (int p = r + 1; p <= flat; ++p) add_lane_merge(r, g0, p, true);
    P.g[P.ngroups++] = g0;
    const int mid = L < r + 6 ? L : r + 6;
    for (int p = flat + 1; p <= mid; ++p) add_merge_bits(P, p - 1, true);
    for (int p = r + 7; p <= L; ++p) {
      Group G{};
      G.r = r;
      for (int m = 0; m < r; ++m) G.v[m] = 1u << (p - 1 - m);
      G.vmirror = p;
      for (int m = 0; m < r; ++m) G.d[G.nsteps++] = 1u << m;  // bits p-1 .. p-r
      P.g[P.ngroups++] = G;
      Group B = blocked_group(r);
      add_lane_merge(r, B, p, false);
      P.g[P.ngroups++] = B;
    }
  } else {
    P.g[P.ngroups++] = g0;
    for (int p = r + 1; p <= L; ++p) add_merge_bits(P, p - 1, true);
  }
  if (L > r) P.g[P.ngroups++] = vector_io ? io_group(L, r) : io_scalar_group(L, r);
  return P;
}

// The last L steps of a phase longer than the tile: strides 2^(L-1) .. 1,
// smaller key to the lower index, on each tile.  With vector I/O the load and
// store layouts hold index bits 0 and 1, so every thread moves 4 consecutive
// keys at a time, and the store layout performs the last two steps; with
// scalar I/O the first merge layout (the top r bits in registers) is already
// the I/O layout.
constexpr Program make_tile_merge(int L, int r, bool vector_io) {
  Program P{};
  P.L = L;
  P.r = r;
  if (vector_io) {
    Group G = io_group(L, r);
    for (int m = 2; m < r; ++m) G.d[G.nsteps++] = 1u << m;
    P.g[P.ngroups++] = G;
    // bits L-r+1 .. 2 in windows of r consecutive bits (the last window may
    // step fewer than r of them); bits 1 and 0 are register bits of the
    // store layout, which performs those two steps itself.
    int top = L - 1 - (r - 2);
    while (top >= 2) {
      const int hi = top > r - 1 ? top : r - 1;  // window hi .. hi-r+1
      Group M{};
      M.r = r;
      for (int m = 0; m < r; ++m) M.v[m] = 1u << (hi - m);
      for (int b = top; b >= 2 && b > hi - r; --b) M.d[M.nsteps++] = 1u << (hi - b);
      P.g[P.ngroups++] = M;
      top = hi - r;
    }
    Group S = io_group(L, r);
    S.d[S.nsteps++] = 2u;
    S.d[S.nsteps++] = 1u;
    P.g[P.ngroups++] = S;
  } else {
    add_merge_bits(P, L - 1, false);
    P.g[P.ngroups++] = io_scalar_group(L, r);
  }
  return P;
}

// All of phase L on each tile whose two halves are each ascending: the
// mirror step on bit L-1, then half-cleaners on bits L-2 .. 0, so the tile
// comes out ascending.  For a sort with 2^(L-1)-key tiles this is phase L in
// one launch instead of a one-step pass and a tile merge.  Loaded and stored
// in the 16-byte I/O layout; the steps run in the layouts of the tile sort's
// longer phases (a virtual layout for the mirror step), one regroup more than
// a merge.
constexpr Program make_tile_phase(int L, int r, bool vector_io) {
  Program P{};
  P.L = L;
  P.r = r;
  const Group io = vector_io ? io_group(L, r) : io_scalar_group(L, r);
  P.g[P.ngroups++] = io;
  add_merge_bits(P, L - 1, true);
  P.g[P.ngroups++] = io;
  return P;
}

// Program kinds: 0 sort, 1 merge (16-byte vector I/O); 2 sort, 3 merge
// (scalar I/O); 4 and 6: the sorts 0 and 2 with lane steps (lane_top
// kLaneTop; see make_tile_sort), for 4-byte keys only (a lane step moves one
// 4-byte word per key); 5 and 7: one whole phase (make_tile_phase) with
// vector and scalar I/O.
constexpr int kLaneTop = 9;
constexpr bool kind_is_vector(int kind) {
  return kind == 0 || kind == 1 || kind == 4 || kind == 5;
}
constexpr bool kind_is_lean(int kind) { return kind == 2 || kind == 3 || kind == 6 || kind == 7; }
constexpr Program make_program(int L, int r, int kind) {
  return kind == 5 || kind == 7 ? make_tile_phase(L, r, kind == 5)
         : (kind & 1) ? make_tile_merge(L, r, kind_is_vector(kind))
                      : make_tile_sort(L, r, kind_is_vector(kind),
                                       kind == 4 || kind == 6 ? kLaneTop : 0);
}

constexpr bool layout_is_vector4(const Group& G) {
  return G.r >= 2 && G.v[0] == 1u && G.v[1] == 2u && G.vmirror == 0;
}

// Total compare-exchange steps a program performs (for checks).
constexpr int program_steps(const Program& P) {
  int s = 0;
  for (int g = 0; g < P.ngroups; ++g) s += P.g[g].nsteps;
  return s;
}

}  // namespace bitonic
