"""Pins for the CPU oracle against facts that do not come from the oracle.

* values the paper prints (sections 3.1, 3.2, 4.2) -- golden fixtures;
* Python's ``sorted`` / numpy's ``sort`` (library routines) on brute-force
  small inputs and on random large ones;
* the 0-1 principle for comparator networks (Knuth, TAOCP vol. 3, 5.3.4):
  a network sorts every input iff it sorts every 0-1 input -- checked
  exhaustively for every n <= 16, power of two or not, both directions;
* the per-phase closed form: after phase p every aligned 2^p block holds the
  sorted keys of the same block of the input.
"""
import itertools

import numpy as np
import pytest

from conftest import read_golden
from oracle import oracle as O
from paper_1506_01446_amd import workloads as W

VARIANTS = (O.STANDARD, O.FLIP, O.FLIP_VIRTUAL)
I32_MIN, I32_MAX = -2**31, 2**31 - 1


def _sorted(keys, ascending):
    return sorted(int(v) for v in keys) if ascending else \
        sorted((int(v) for v in keys), reverse=True)


# -- values the paper prints -------------------------------------------------

def test_sec3_1_worked_bitonic_sequences(oracle_lib):
    g = dict(ln.split(":") for ln in read_golden("sec3_1_bitonic_sequences.txt"))
    merged = [int(v) for v in g["merged"].split()]
    for name in ("rise_fall", "rotated"):
        seq = [int(v) for v in g[name].split()]
        # bitonic: some rotation rises then falls
        assert any(
            (lambda r: r[: r.index(max(r)) + 1] == sorted(r[: r.index(max(r)) + 1])
             and r[r.index(max(r)):] == sorted(r[r.index(max(r)):], reverse=True))(
                seq[s:] + seq[:s]) for s in range(len(seq)))
        assert list(O.bitonic_merge_i32(seq)) == merged
        assert merged == sorted(seq)


def test_sec3_1_network_n8_counts(oracle_lib):
    g = dict(ln.split(":") for ln in read_golden("sec3_1_network_n8.txt"))
    n = int(g["n"])
    per_phase = [int(v) for v in g["steps_per_phase"].split()]
    assert len(per_phase) == int(g["phases"])
    seen = []
    for variant in VARIANTS:
        seen.clear()
        _, steps, cmps = O.bitonic_i32(np.arange(n)[::-1], True, variant,
                                       hook=lambda p, s, x: seen.append((p, s)))
        assert steps == int(g["steps"]) == sum(per_phase)
        assert cmps == int(g["cmp_total"])
        assert [sum(1 for p, _ in seen if p == ph) for ph in range(1, 4)] == per_phase
        for ph, nsteps in enumerate(per_phase, start=1):
            for st in range(1, nsteps + 1):
                assert len(O.step_pairs(n, variant, ph, st)) == int(g["cmp_per_step"])


def test_sec3_2_closed_forms(oracle_lib):
    rows = [tuple(int(v) for v in ln.split()) for ln in read_golden("sec3_2_counts.txt")]
    for k, rounds, cmps in rows:
        assert rounds == k * (k + 1) // 2
        assert cmps == (2**k) * k * (k + 1) // 4
    for k in range(0, 15):
        n = 2**k
        for variant in VARIANTS:
            _, steps, cmps = O.bitonic_i32(W.uniform_i32(k, n), True, variant)
            assert steps == k * (k + 1) // 2
            assert cmps == n * k * (k + 1) // 4
    # materialised padding runs the full network of N = 2^k; the virtual
    # arrangement skips exactly the comparators reaching past n
    for n in (3, 5, 1000, 1025):
        k = (n - 1).bit_length()
        _, s1, c1 = O.bitonic_i32(W.uniform_i32(n, n), True, O.FLIP)
        _, s2, c2 = O.bitonic_i32(W.uniform_i32(n, n), True, O.FLIP_VIRTUAL)
        assert s1 == s2 == k * (k + 1) // 2
        assert c1 == 2**k * k * (k + 1) // 4 and c2 < c1


def test_sec4_2_register_pairs(oracle_lib):
    rows = [tuple(int(v) for v in ln.split()) for ln in read_golden("sec4_2_register_pairs.txt")]
    held = {0, 2, 4, 6}
    for phase, step in {(r[0], r[1]) for r in rows}:
        pairs = [(lo, hi) for lo, hi, _ in O.step_pairs(8, O.STANDARD, phase, step)
                 if lo in held and hi in held]
        assert sorted(pairs) == sorted((r[2], r[3]) for r in rows
                                       if (r[0], r[1]) == (phase, step))
    # those two steps only ever pair addresses inside {0,2,4,6} or {1,3,5,7}
    for step in (1, 2):
        for lo, hi, _ in O.step_pairs(8, O.STANDARD, 3, step):
            assert (lo in held) == (hi in held)


def test_step_pairs_shapes(oracle_lib):
    # standard network: partner = i xor stride, direction by bit p of i
    for lo, hi, up in O.step_pairs(16, O.STANDARD, 3, 2):
        assert hi == lo ^ 2 and up == ((lo & 8) == 0)
    # flip network: first step pairs mirror images inside the 2^p block
    for lo, hi, up in O.step_pairs(16, O.FLIP, 3, 1):
        assert hi == lo ^ 7 and up
    for lo, hi, up in O.step_pairs(16, O.FLIP, 3, 3):
        assert hi == lo ^ 1 and up


# -- brute force against library sorts ----------------------------------------

@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("ascending", [True, False])
def test_all_permutations(oracle_lib, variant, ascending):
    for n in range(0, 9):
        perms = np.array(list(itertools.permutations(range(n))), dtype=np.int32)
        if n == 0:
            out, _, _ = O.bitonic_i32(np.zeros(0, np.int32), ascending, variant)
            assert out.size == 0
            continue
        out = O.bitonic_batch_i32(perms, ascending, variant)
        want = np.arange(n, dtype=np.int32)
        if not ascending:
            want = want[::-1]
        assert (out == want).all(), (n, variant, ascending)


@pytest.mark.parametrize("variant", VARIANTS)
def test_all_words_with_repeats(oracle_lib, variant):
    for n in range(1, 10):
        words = np.array(list(itertools.product((-1, 0, 1), repeat=n)), dtype=np.int32)
        for ascending in (True, False):
            out = O.bitonic_batch_i32(words, ascending, variant)
            want = np.sort(words, axis=1)
            if not ascending:
                want = want[:, ::-1]
            assert (out == want).all(), (n, variant, ascending)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("ascending", [True, False])
def test_zero_one_principle(oracle_lib, variant, ascending):
    """Every 0-1 input of every length n <= 16 is sorted."""
    for n in range(1, 17):
        codes = np.arange(2**n, dtype=np.int64)
        bits = ((codes[:, None] >> np.arange(n)) & 1).astype(np.int32)
        out = O.bitonic_batch_i32(bits, ascending, variant)
        ones = bits.sum(axis=1)
        pos = np.arange(n)[None, :]
        want = (pos >= (n - ones)[:, None]) if ascending else (pos < ones[:, None])
        assert (out == want.astype(np.int32)).all(), (n, variant, ascending)


def test_signed_extremes(oracle_lib):
    base = [I32_MAX, I32_MIN, -1, 0, 1, I32_MAX, I32_MIN, 7, -7]
    for n in range(1, len(base) + 1):
        keys = np.array(base[:n], dtype=np.int32)
        for ascending in (True, False):
            want = _sorted(keys, ascending)
            assert list(O.sort_i32(keys, ascending)) == want
            for variant in VARIANTS:
                out, _, _ = O.bitonic_i32(keys, ascending, variant)
                assert list(out) == want, (n, variant, ascending)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 255, 256, 257, 1000, 4096, 5000, 65536])
def test_random_against_numpy(oracle_lib, n):
    keys = W.uniform_i32(W.SEED_BASE + n, n)
    for ascending in (True, False):
        want = np.sort(keys)
        if not ascending:
            want = want[::-1]
        assert (O.sort_i32(keys, ascending) == want).all()
        for variant in VARIANTS:
            out, _, _ = O.bitonic_i32(keys, ascending, variant)
            assert (out == want).all(), (variant, ascending)


@pytest.mark.parametrize("kind", W.KINDS)
def test_distributions(oracle_lib, kind):
    keys = W.make_keys(kind, W.SEED_BASE + 10, 3000)
    for ascending in (True, False):
        want = np.sort(keys) if ascending else np.sort(keys)[::-1]
        out, _, _ = O.bitonic_i32(keys, ascending, O.FLIP_VIRTUAL)
        assert (out == want).all()


# -- per-phase closed form ------------------------------------------------------

@pytest.mark.parametrize("n", [64, 100, 1024, 1500])
def test_per_phase_blocks(oracle_lib, n):
    keys = W.uniform_i32(W.SEED_BASE + 99, n)
    N = 1 << (n - 1).bit_length()
    padded = np.full(N, I32_MAX, dtype=np.int32)
    padded[:n] = keys
    for variant in VARIANTS:
        states = {}

        def hook(p, s, x):
            if s == p:
                states[p] = x

        O.bitonic_i32(keys, True, variant, hook=hook)
        k = N.bit_length() - 1
        assert sorted(states) == list(range(1, k + 1))
        for p, x in states.items():
            B = 1 << p
            src = padded if variant != O.FLIP_VIRTUAL else keys
            for b0 in range(0, len(x), B):
                blk = np.sort(src[b0:b0 + B])
                if variant == O.STANDARD and p < k and (b0 & B):
                    blk = blk[::-1]
                assert (x[b0:b0 + B] == blk).all(), (variant, p, b0)


# -- segmented ------------------------------------------------------------------

def test_segmented(oracle_lib):
    lens = np.array([0, 1, 2, 3, 0, 8, 9, 100, 1, 0, 513], dtype=np.int64)
    off = W.offsets_from_lengths(lens)
    keys = W.uniform_i32(5, int(off[-1]))
    for ascending in (True, False):
        got = O.sort_segmented_i32(keys, off, ascending)
        net = O.bitonic_segmented_i32(keys, off, ascending)
        for s in range(len(lens)):
            seg = np.sort(keys[off[s]:off[s + 1]])
            if not ascending:
                seg = seg[::-1]
            assert (got[off[s]:off[s + 1]] == seg).all()
            assert (net[off[s]:off[s + 1]] == seg).all()


def test_bad_arguments(oracle_lib):
    with pytest.raises(ValueError):
        O.bitonic_merge_i32([3, 1, 2])
    with pytest.raises(ValueError):
        O.sort_segmented_i32([1, 2, 3], [0, 5])
    with pytest.raises(ValueError):
        O.step_pairs(8, O.STANDARD, 4, 1)


@pytest.mark.parametrize("threads", [1, 2, 3, 7, 16])
def test_parallel_sort_baseline(oracle_lib, threads):
    """The all-cores CPU baseline (chunks sorted in parallel, merged pairwise)
    gives numpy's sort: sizes below, at and above the thread count, ragged
    chunks, both directions."""
    from oracle import oracle as O
    for n in (0, 1, 2, threads - 1, threads, threads + 1, 1000, 65537, 300001):
        if n < 0:
            continue
        keys = W.uniform_i32(n + 31 * threads, n)
        keys[: n // 3] = keys[n // 3: 2 * (n // 3)] if n >= 3 else keys[: n // 3]  # duplicates
        for asc in (True, False):
            got = O.sort_i32_parallel(keys, asc, threads)
            want = np.sort(keys) if asc else np.sort(keys)[::-1]
            assert np.array_equal(got, want), (n, threads, asc)
