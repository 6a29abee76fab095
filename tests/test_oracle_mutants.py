"""The oracle's pins catch plausible mistakes.

Each mutant is the oracle source rebuilt with one planted mistake (a dropped
step, a wrong partner index, a lost direction alternation, an unsigned
compare, wrong padding).  Every mutant must fail at least one pin; the clean
build must pass them all.  Mistakes are planted in the oracle only, on the
CPU.
"""
import numpy as np
import pytest

from oracle import build_oracle
from oracle import oracle as O
from paper_1506_01446_amd import workloads as W

I32_MAX = 2**31 - 1


def _pin_zero_one(lib):
    for variant in (O.STANDARD, O.FLIP, O.FLIP_VIRTUAL):
        for n in range(1, 13):
            codes = np.arange(2**n, dtype=np.int64)
            bits = ((codes[:, None] >> np.arange(n)) & 1).astype(np.int32)
            for asc in (True, False):
                out = O.bitonic_batch_i32(bits, asc, variant, lib=lib)
                want = np.sort(bits, axis=1)
                if not asc:
                    want = want[:, ::-1]
                if not (out == want).all():
                    return False
    return True


def _pin_signed_random(lib):
    keys = W.uniform_i32(123, 777)
    keys[:3] = [I32_MAX, -2**31, -1]
    for variant in (O.STANDARD, O.FLIP, O.FLIP_VIRTUAL):
        out, _, _ = O.bitonic_i32(keys, True, variant, lib=lib)
        if not (out == np.sort(keys)).all():
            return False
    return (O.sort_i32(keys, True, lib=lib) == np.sort(keys)).all()


def _pin_counts(lib):
    for k in range(1, 9):
        for variant in (O.STANDARD, O.FLIP):
            _, steps, cmps = O.bitonic_i32(np.arange(2**k), True, variant, lib=lib)
            if steps != k * (k + 1) // 2 or cmps != 2**k * k * (k + 1) // 4:
                return False
    return True


def _pin_negative_padding(lib):
    # non-power-of-two inputs whose keys are all negative: wrong sentinels
    # would be pulled into the result
    keys = -np.arange(1, 12, dtype=np.int32)
    for variant in (O.STANDARD, O.FLIP):
        for asc in (True, False):
            out, _, _ = O.bitonic_i32(keys, asc, variant, lib=lib)
            want = np.sort(keys) if asc else np.sort(keys)[::-1]
            if not (out == want).all():
                return False
    return True


def _pin_f32_total_order(lib):
    from test_oracle_keytypes import TOTAL_ORDER
    want = np.array(TOTAL_ORDER, dtype=np.uint32)
    got = O.sort_keys(want[::-1].view(np.float32), O.KEY_F32, True, lib=lib).view(np.uint32)
    return bool(np.array_equal(got, want))


def _pin_keys64(lib):
    keys = W.uniform_i64(8, 3001)
    keys[:2] = [2**63 - 1, -2**63]
    return bool(np.array_equal(O.sort_keys64(keys, O.KEY_I64, True, lib=lib), np.sort(keys)))


def _pin_f64_total_order(lib):
    from test_oracle_wide import TOTAL_ORDER64
    want = np.array(TOTAL_ORDER64, dtype=np.uint64)
    got = O.sort_keys64(want[::-1].view(np.float64), O.KEY_F64, True, lib=lib).view(np.uint64)
    return bool(np.array_equal(got, want))


def _pin_pairs(lib):
    keys = (W.uniform_i32(9, 2000).astype(np.int64) % 17).astype(np.int32)
    values = W.uniform_i32(10, 2000)
    k, v = O.sort_pairs(keys, values, O.KEY_I32, True, lib=lib)
    order = np.lexsort((values, keys))
    return bool(np.array_equal(k, keys[order]) and np.array_equal(v, values[order]))


PINS = (_pin_zero_one, _pin_signed_random, _pin_counts, _pin_negative_padding,
        _pin_f32_total_order, _pin_keys64, _pin_f64_total_order, _pin_pairs)


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("oracle_mutants"))


def test_clean_oracle_passes_all_pins(oracle_lib):
    assert oracle_lib.oracle_mutant_id() == 0
    for pin in PINS:
        assert pin(oracle_lib), pin.__name__


@pytest.mark.parametrize("mutant", sorted(build_oracle.MUTANTS))
def test_mutant_is_caught(mutant, mutant_dir):
    lib = O.load(build_oracle.build_mutant(mutant, mutant_dir))
    assert lib.oracle_mutant_id() == mutant
    failed = [pin.__name__ for pin in PINS if not pin(lib)]
    assert failed, f"mutant {mutant} ({build_oracle.MUTANTS[mutant]}) passed every pin"
