"""Pins for the oracle's other 32-bit key types (uint32, float32 in IEEE
754-2008 totalOrder): numpy's sort where it is defined the same way, and
hand-written cases from the definition of totalOrder."""
import numpy as np
import pytest

from oracle import build_oracle
from oracle import oracle as O
from paper_1506_01446_amd import workloads as W


def _f32(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32)


def test_u32_against_numpy(oracle_lib):
    for n in (0, 1, 7, 1000, 65537):
        keys = W.uniform_i32(n + 5, n).view(np.uint32)
        for asc in (True, False):
            want = np.sort(keys) if asc else np.sort(keys)[::-1]
            assert np.array_equal(O.sort_keys(keys, O.KEY_U32, asc), want)


def test_f32_against_numpy_without_nans_or_zeros(oracle_lib):
    rng_bits = W.uniform_i32(11, 50000).view(np.uint32)
    keys = _f32(rng_bits)
    keys = keys[np.isfinite(keys) & (keys != 0)]
    for asc in (True, False):
        want = np.sort(keys) if asc else np.sort(keys)[::-1]
        got = O.sort_keys(keys, O.KEY_F32, asc)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


# IEEE 754-2008 5.10 totalOrder, written out: -qNaN < -sNaN < -inf < negative
# normals (larger magnitude first) < negative subnormals < -0 < +0 < ... <
# +inf < +sNaN < +qNaN.
TOTAL_ORDER = [
    0xFFC00001,  # -qNaN with payload 1
    0xFFC00000,  # -qNaN
    0xFF800001,  # -sNaN
    0xFF800000,  # -inf
    0xC0000000,  # -2
    0xBF800000,  # -1
    0x80000001,  # -smallest subnormal
    0x80000000,  # -0
    0x00000000,  # +0
    0x00000001,  # +smallest subnormal
    0x3F800000,  # +1
    0x40000000,  # +2
    0x7F800000,  # +inf
    0x7F800001,  # +sNaN
    0x7FC00000,  # +qNaN
    0x7FC00001,  # +qNaN with payload 1
]


def test_f32_total_order_cases(oracle_lib):
    want = np.array(TOTAL_ORDER, dtype=np.uint32)
    for seed in range(5):
        perm = np.argsort(W.uniform_i32(seed, len(want)))
        got = O.sort_keys(_f32(want[perm]), O.KEY_F32, True).view(np.uint32)
        assert np.array_equal(got, want)
        got = O.sort_keys(_f32(want[perm]), O.KEY_F32, False).view(np.uint32)
        assert np.array_equal(got, want[::-1])


def test_segmented_keys(oracle_lib):
    lens = np.array([3, 0, 100, 1, 17], dtype=np.int64)
    off = W.offsets_from_lengths(lens)
    bits = W.uniform_i32(3, int(off[-1])).view(np.uint32)
    for kt in (O.KEY_I32, O.KEY_U32, O.KEY_F32):
        got = O.sort_segmented_keys(bits.view(O._KEY_DTYPES[kt]), off, kt, False)
        for s in range(len(lens)):
            seg = bits[off[s]:off[s + 1]].view(O._KEY_DTYPES[kt])
            want = O.sort_keys(seg, kt, False)
            assert np.array_equal(got[off[s]:off[s + 1]].view(np.uint32), want.view(np.uint32))


def test_f32_mutant_is_caught(tmp_path):
    lib = O.load(build_oracle.build_mutant(7, str(tmp_path)))
    want = np.array(TOTAL_ORDER, dtype=np.uint32)
    got = O.sort_keys(_f32(want[::-1]), O.KEY_F32, True, lib=lib).view(np.uint32)
    assert not np.array_equal(got, want)
