// CPU emulation of the tile programs of the HIP library (program.hpp), for
// host-side tests: runs a tile through the same layouts, register steps and
// LDS regroupings the tile kernels perform, one simulated thread at a time,
// and counts LDS bank conflicts of the regroupings.  It includes only the
// library's program description, never the oracle.
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../paper_1506_01446_amd/csrc/program.hpp"

using namespace bitonic;

static uint32_t deposit_rt(uint32_t mask, uint32_t t) {
  uint32_t out = 0;
  int k = 0;
  for (int b = 0; b < 32; ++b)
    if ((mask >> b) & 1u) {
      out |= ((t >> k) & 1u) << b;
      ++k;
    }
  return out;
}

// LDS position of slot j of thread t in layout G: the padded position of the
// slot's real index (virtual layouts mirror the upper half of each block).
static uint32_t lds_addr(const Group& G, int L, uint32_t t, uint32_t j) {
  uint32_t base = deposit_rt(free_mask(G, L), t);
  if (slot_mirrored(G, j)) base ^= mirror_mask(G) & free_mask(G, L);
  return lds_pad(base, G.r) + lds_pad(real_off(G, j), G.r);
}

// Real tile index of slot j of thread t (checks the additive address form).
static uint32_t real_index(const Group& G, int L, uint32_t t, uint32_t j) {
  const uint32_t v = deposit_rt(free_mask(G, L), t) | goff(G, j);
  if (G.vmirror > 0 && ((v >> (G.vmirror - 1)) & 1u)) return v ^ mirror_mask(G);
  return v;
}

static Program make(int L, int r, int kind) {
  return make_program(L, r, kind);
}

// Every layout's basis: r distinct single index bits below L; every step a
// nonzero register mask.
static bool layouts_valid(const Program& P, int L) {
  for (int g = 0; g < P.ngroups; ++g) {
    const Group& G = P.g[g];
    if (G.nsteps > kMaxSteps) return false;
    uint32_t seen = 0;
    for (int m = 0; m < G.r; ++m) {
      const uint32_t v = G.v[m];
      if (v == 0 || (v & (v - 1)) || v >= (1u << L) || (seen & v)) return false;
      seen |= v;
    }
    for (int s = 0; s < G.nsteps; ++s) {
      const uint32_t D = G.d[s];
      if (D == 0 || step_reg(D) >= (1u << G.r) || step_lane(D) >= 64u) return false;
    }
  }
  return true;
}

extern "C" {

// Returns the number of compare-exchange steps performed, or -1 on error
// (e.g. an LDS regrouping that is not a permutation).
int emulate_tile(int L, int r, int kind, int32_t* tile, uint32_t valid) {
  const Program P = make(L, r, kind);
  if (!layouts_valid(P, L)) return -1;
  const uint32_t T = 1u << L, NT = 1u << (L - r), R = 1u << r;
  const int32_t PAD = 0x7FFFFFFF;
  std::vector<int32_t> x(size_t(NT) * R);
  {
    const Group& G = P.g[0];
    for (uint32_t t = 0; t < NT; ++t) {
      const uint32_t base = deposit_rt(free_mask(G, L), t);
      for (uint32_t j = 0; j < R; ++j) {
        const uint32_t i = base ^ goff(G, j);
        if (i >= T) return -1;
        x[t * R + j] = i < valid ? tile[i] : PAD;
      }
    }
  }
  int steps = 0;
  const uint32_t W = lds_words(L, r);
  std::vector<int32_t> lds(W);
  std::vector<int> hit(W);
  for (int g = 0; g < P.ngroups; ++g) {
    const Group& G = P.g[g];
    if (g > 0) {
      const Group& A = P.g[g - 1];
      std::fill(hit.begin(), hit.end(), 0);
      for (uint32_t t = 0; t < NT; ++t) {
        for (uint32_t j = 0; j < R; ++j) {
          const uint32_t a = lds_addr(A, L, t, j);
          if (a >= W || a != lds_pad(real_index(A, L, t, j), r)) return -1;
          lds[a] = x[t * R + j];
          hit[a]++;
        }
      }
      uint32_t filled = 0;
      for (uint32_t a = 0; a < W; ++a) {
        if (hit[a] > 1) return -1;
        filled += hit[a];
      }
      if (filled != T) return -1;
      for (uint32_t t = 0; t < NT; ++t)
        for (uint32_t j = 0; j < R; ++j) {
          const uint32_t a = lds_addr(G, L, t, j);
          if (a != lds_pad(real_index(G, L, t, j), r)) return -1;
          x[t * R + j] = lds[a];
        }
    }
    for (int s = 0; s < G.nsteps; ++s) {
      const uint32_t D = G.d[s];
      if (step_lane(D) == 0) {
        for (uint32_t t = 0; t < NT; ++t)
          for (uint32_t j = 0; j < R; ++j) {
            const uint32_t jj = j ^ D;
            if (j >= jj) continue;
            int32_t& lo = slot_is_lower(G, j, D) ? x[t * R + j] : x[t * R + jj];
            int32_t& hi = slot_is_lower(G, j, D) ? x[t * R + jj] : x[t * R + j];
            const int32_t a = std::min(lo, hi), b = std::max(lo, hi);
            lo = a;
            hi = b;
          }
      } else {
        // lane step: slot j of thread t meets slot j ^ DR of thread t ^ M (the
        // same 64-lane wave); the thread with lane bit highbit(M) set keeps
        // the maximum.  Both ends must be the same pair of real indices seen
        // from either side, one step of the network apart (i ^ partner has
        // its highest bit where the lane bit says).
        const uint32_t M = step_lane(D), DR = step_reg(D);
        const int hb = highbit(M);
        std::vector<int32_t> y(x);
        for (uint32_t t = 0; t < NT; ++t) {
          const uint32_t tp = t ^ M;
          if (tp >= NT || tp / 64 != t / 64) return -1;
          for (uint32_t j = 0; j < R; ++j) {
            const uint32_t jj = j ^ DR;
            const uint32_t i = real_index(G, L, t, j), ip = real_index(G, L, tp, jj);
            const bool upper = ((t >> hb) & 1u) != 0;
            if ((i > ip) != upper) return -1;
            const int32_t a = x[t * R + j], b = x[tp * R + jj];
            y[t * R + j] = upper ? std::max(a, b) : std::min(a, b);
          }
        }
        x.swap(y);
      }
      ++steps;
    }
  }
  {
    const Group& G = P.g[P.ngroups - 1];
    for (uint32_t t = 0; t < NT; ++t) {
      const uint32_t base = deposit_rt(free_mask(G, L), t);
      for (uint32_t j = 0; j < R; ++j) {
        const uint32_t i = base ^ goff(G, j);
        if (i < valid) tile[i] = x[t * R + j];
      }
    }
  }
  return steps;
}

// Worst number of lanes of one group of `lanes` consecutive lanes that hit
// the same LDS bank (of `banks`, in units of one LDS word) in any access of
// any regrouping of the program.  32 lanes over 32 banks models 4-byte words
// (a half-wave per access cycle); 16 lanes over 32 banks models 8-byte words
// (a quarter-wave of 128 bytes per cycle, each word on a pair of banks).
int worst_bank_conflict_lanes(int L, int r, int kind, int banks, int lanes) {
  const Program P = make(L, r, kind);
  if (!layouts_valid(P, L)) return -1;
  const uint32_t NT = 1u << (L - r), R = 1u << r;
  int worst = 0;
  for (int g = 1; g < P.ngroups; ++g) {
    for (int side = 0; side < 2; ++side) {
      const Group& G = side == 0 ? P.g[g - 1] : P.g[g];
      for (uint32_t w0 = 0; w0 < NT; w0 += (uint32_t)lanes)
        for (uint32_t j = 0; j < R; ++j) {
          std::vector<int> cnt(banks, 0);
          for (uint32_t t = w0; t < w0 + (uint32_t)lanes && t < NT; ++t) {
            const uint32_t a = lds_addr(G, L, t, j);
            worst = std::max(worst, ++cnt[a % banks]);
          }
        }
    }
  }
  return worst;
}

int worst_bank_conflict(int L, int r, int kind, int banks) {
  return worst_bank_conflict_lanes(L, r, kind, banks, 32);
}

int program_groups(int L, int r, int kind) { return make(L, r, kind).ngroups; }

// The regroups the kernels synchronise per wave only (regroup_in_wave of
// program.hpp) against an exhaustive check: a regroup keeps every key in its
// wave if each real index a thread of wave w holds in the source layout is
// held by a thread of wave w in the target layout (64-lane waves, thread t in
// wave t / 64).  Returns -1 if the library's test calls a regroup in-wave
// that is not; else writes the number of regroups the exhaustive check finds
// in-wave to *exact and returns the number the library's test finds.
int in_wave_regroups(int L, int r, int kind, int* exact) {
  const Program P = make(L, r, kind);
  if (!layouts_valid(P, L)) return -1;
  const uint32_t NT = 1u << (L - r), R = 1u << r;
  int lib = 0, truth = 0;
  for (int g = 1; g < P.ngroups; ++g) {
    const Group& A = P.g[g - 1];
    const Group& B = P.g[g];
    // owner thread of every real index in layout B
    std::vector<uint32_t> owner(size_t(1) << L);
    for (uint32_t t = 0; t < NT; ++t)
      for (uint32_t j = 0; j < R; ++j) owner[real_index(B, L, t, j)] = t;
    bool stays = true;
    for (uint32_t t = 0; t < NT && stays; ++t)
      for (uint32_t j = 0; j < R; ++j)
        if (owner[real_index(A, L, t, j)] / 64 != t / 64) {
          stays = false;
          break;
        }
    const bool flagged = regroup_in_wave(A, B, L);
    if (flagged && !stays) return -1;
    lib += flagged;
    truth += stays;
  }
  *exact = truth;
  return lib;
}

}  // extern "C"
