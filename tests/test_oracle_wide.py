"""Pins for the oracle's 8-byte key types and its key-value sort.

* int64 / uint64: numpy's sort (a library routine, same order by definition).
* float64: numpy's sort on finite non-zero values, and the special values of
  IEEE 754-2008 5.10 totalOrder written out by hand.
* pairs: numpy's lexsort (key, then value) and, with values 0..n-1, numpy's
  stable argsort; brute force over every arrangement of small inputs (the
  order is unique, so every arrangement must give the same result).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from paper_1506_01446_amd import workloads as W


def _i64_keys(seed, n):
    keys = W.uniform_i64(seed, n)
    if n >= 4:
        keys[:4] = [2**63 - 1, -2**63, -1, 0]
    return keys


def test_i64_and_u64_against_numpy(oracle_lib):
    for n in (0, 1, 7, 1000, 65537):
        keys = _i64_keys(n + 3, n)
        for asc in (True, False):
            want = np.sort(keys) if asc else np.sort(keys)[::-1]
            assert np.array_equal(O.sort_keys64(keys, O.KEY_I64, asc), want)
            u = keys.view(np.uint64)
            want = np.sort(u) if asc else np.sort(u)[::-1]
            assert np.array_equal(O.sort_keys64(u, O.KEY_U64, asc), want)


def test_i64_high_words_tie(oracle_lib):
    # keys that agree in their high 32 bits are ordered by the low ones
    hi = np.int64(5) << np.int64(32)
    keys = np.array([hi + 3, hi - 7, hi + 0x7FFFFFFF, hi + 1, -hi + 2, -hi - 2], dtype=np.int64)
    assert np.array_equal(O.sort_keys64(keys, O.KEY_I64), np.sort(keys))


def test_f64_against_numpy_without_nans_or_zeros(oracle_lib):
    keys = W.uniform_i64(21, 50000).view(np.float64)
    keys = keys[np.isfinite(keys) & (keys != 0)]
    for asc in (True, False):
        want = np.sort(keys) if asc else np.sort(keys)[::-1]
        got = O.sort_keys64(keys, O.KEY_F64, asc)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


# IEEE 754-2008 5.10 totalOrder on binary64, written out: -qNaN < -sNaN <
# -inf < negative normals (larger magnitude first) < negative subnormals <
# -0 < +0 < positive subnormals < positive normals < +inf < +sNaN < +qNaN.
TOTAL_ORDER64 = [
    0xFFF8000000000001,  # -qNaN, payload 1
    0xFFF8000000000000,  # -qNaN
    0xFFF0000000000001,  # -sNaN
    0xFFF0000000000000,  # -inf
    0xFFEFFFFFFFFFFFFF,  # -max finite
    0xC000000000000000,  # -2
    0xBFF0000000000000,  # -1
    0x8010000000000000,  # -min normal
    0x800FFFFFFFFFFFFF,  # -max subnormal
    0x8000000000000001,  # -min subnormal
    0x8000000000000000,  # -0
    0x0000000000000000,  # +0
    0x0000000000000001,  # +min subnormal
    0x000FFFFFFFFFFFFF,  # +max subnormal
    0x0010000000000000,  # +min normal
    0x3FF0000000000000,  # +1
    0x4000000000000000,  # +2
    0x7FEFFFFFFFFFFFFF,  # +max finite
    0x7FF0000000000000,  # +inf
    0x7FF0000000000001,  # +sNaN
    0x7FF8000000000000,  # +qNaN
    0x7FF8000000000001,  # +qNaN, payload 1
]


def test_f64_total_order_special_values(oracle_lib):
    want = np.array(TOTAL_ORDER64, dtype=np.uint64)
    for perm_seed in range(5):
        order = np.argsort(W.uniform_i32(perm_seed, want.size), kind="stable")
        got = O.sort_keys64(want[order].view(np.float64), O.KEY_F64, True).view(np.uint64)
        assert np.array_equal(got, want)
        got = O.sort_keys64(want[order].view(np.float64), O.KEY_F64, False).view(np.uint64)
        assert np.array_equal(got, want[::-1])


def _pairs_input(seed, n, distinct=64):
    keys = (W.uniform_i32(seed, n).astype(np.int64) % distinct).astype(np.int32) - distinct // 2
    values = W.uniform_i32(seed + 1, n)
    return keys, values


def test_pairs_against_lexsort(oracle_lib):
    for n in (0, 1, 2, 9, 1000, 40001):
        keys, values = _pairs_input(n + 40, n)
        for asc in (True, False):
            order = np.lexsort((values, keys if asc else -keys.astype(np.int64)))
            k, v = O.sort_pairs(keys, values, O.KEY_I32, asc)
            assert np.array_equal(k, keys[order]) and np.array_equal(v, values[order])


def test_pairs_unsigned_and_float_keys_against_lexsort(oracle_lib):
    n = 20000
    keys, values = _pairs_input(77, n, distinct=1000)
    u = keys.view(np.uint32)
    for asc in (True, False):
        order = np.lexsort((values, u if asc else (np.uint64(2**32 - 1) - u.astype(np.uint64))))
        k, v = O.sort_pairs(u, values, O.KEY_U32, asc)
        assert np.array_equal(k, u[order]) and np.array_equal(v, values[order])
    f = (keys.astype(np.float32) * np.float32(0.25)) + np.float32(0.125)  # finite, non-zero
    for asc in (True, False):
        order = np.lexsort((values, f if asc else -f))
        k, v = O.sort_pairs(f, values, O.KEY_F32, asc)
        assert np.array_equal(k.view(np.uint32), f[order].view(np.uint32))
        assert np.array_equal(v, values[order])


def test_pairs_with_indices_are_a_stable_argsort(oracle_lib):
    n = 30000
    keys, _ = _pairs_input(5, n, distinct=300)
    idx = np.arange(n, dtype=np.int32)
    _, v = O.sort_pairs(keys, idx, O.KEY_I32, True)
    assert np.array_equal(v, np.argsort(keys, kind="stable"))
    _, v = O.sort_pairs(keys, idx, O.KEY_I32, False)
    assert np.array_equal(v, np.argsort(-keys.astype(np.int64), kind="stable"))


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_pairs_brute_force(oracle_lib, n):
    """Every arrangement of a multiset of pairs (equal keys, equal values and
    equal pairs included) sorts to one result, ordered by (key, value)."""
    keys = np.array([1, -1, 1, 0, 1, -1][:n], dtype=np.int32)
    values = np.array([2, 2, -3, 2, 2, 7][:n], dtype=np.int32)
    for asc in (True, False):
        results = set()
        for perm in itertools.permutations(range(n)):
            p = list(perm)
            k, v = O.sort_pairs(keys[p], values[p], O.KEY_I32, asc)
            results.add((tuple(k.tolist()), tuple(v.tolist())))
        assert len(results) == 1
        (k, v), = results
        sign = 1 if asc else -1
        seq = [(sign * a, b) for a, b in zip(k, v)]
        assert seq == sorted(seq)
