"""Host-side checks of the tile programs the HIP kernels are generated from.

The tile kernels are compile-time programs (program.hpp): register layouts,
compare-exchange steps and LDS regroupings.  A CPU emulator runs a tile
through the same program; the result must be the sorted tile (tile sort) or
the merged tile (tile merge), with absent keys past ``valid`` left alone.
Expected values come from numpy's sort, not from the library.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1506_01446_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("emu") / "libemu.so")
    subprocess.run(["g++", "-O2", "-std=c++20", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "cpu_program_emulator.cpp")], check=True)
    lib = ctypes.CDLL(out)
    lib.emulate_tile.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_uint32]
    lib.emulate_tile.restype = ctypes.c_int
    lib.worst_bank_conflict.argtypes = [ctypes.c_int] * 4
    lib.worst_bank_conflict.restype = ctypes.c_int
    lib.worst_bank_conflict_lanes.argtypes = [ctypes.c_int] * 5
    lib.worst_bank_conflict_lanes.restype = ctypes.c_int
    lib.program_groups.argtypes = [ctypes.c_int] * 3
    lib.program_groups.restype = ctypes.c_int
    lib.in_wave_regroups.argtypes = [ctypes.c_int] * 3 + [ctypes.POINTER(ctypes.c_int)]
    lib.in_wave_regroups.restype = ctypes.c_int
    return lib


def _run(emu, L, r, kind, tile, valid):
    x = np.ascontiguousarray(tile, dtype=np.int32).copy()
    steps = emu.emulate_tile(L, r, kind, x.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), valid)
    assert steps >= 0, "program is not a permutation of the tile"
    return x, steps


@pytest.mark.parametrize("L", [11, 12, 13, 14, 15])
def test_tile_sort_program(emu, L):
    T = 1 << L
    for seed in range(3):
        keys = W.uniform_i32(seed, T)
        out, steps = _run(emu, L, 5, 0, keys, T)
        assert steps == L * (L + 1) // 2
        assert (out == np.sort(keys)).all()
    for kind in ("sorted", "reverse", "distinct16", "equal"):
        keys = W.make_keys(kind, 7, T)
        out, _ = _run(emu, L, 5, 0, keys, T)
        assert (out == np.sort(keys)).all()


@pytest.mark.parametrize("L", list(range(5, 14)))
def test_scalar_io_lane_step_program(emu, L):
    """The scalar-I/O sort of 4-byte keys with lane steps (kind 6: segments
    and arrays off a 16-byte boundary): sorted, full and partial tiles; below
    a full wave of lanes (L < 11) it is the plain program."""
    T = 1 << L
    for valid in sorted({T, T - 1, T // 2 + 3, 1}):
        keys = W.uniform_i32(L * 13 + valid, T)
        out, steps = _run(emu, L, 5, 6, keys, valid)
        assert steps == L * (L + 1) // 2
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()
    if L < 11:
        assert emu.program_groups(L, 5, 6) == emu.program_groups(L, 5, 2)
    else:
        assert emu.program_groups(L, 5, 6) < emu.program_groups(L, 5, 2)
    if L > 5:
        assert emu.worst_bank_conflict(L, 5, 6, 32) == 1


@pytest.mark.parametrize("L", [11, 12, 13, 14, 15])
def test_tile_sort_lane_step_program(emu, L):
    """The sort program whose steps on the blocked layout's lane bits run as
    lane steps (cross-lane compare-exchanges, kind 4): every lane step pairs
    the right indices, the tile comes out sorted, full and partial; phases up
    to 9 need no regroup, 10 and 11 regroup through LDS as before, longer
    ones take two regroups."""
    T = 1 << L
    for valid in (T, T - 1, T // 2 + 7, 3):
        keys = W.uniform_i32(L * 7 + valid, T)
        out, steps = _run(emu, L, 5, 4, keys, valid)
        assert steps == L * (L + 1) // 2
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()
    for kind in ("reverse", "distinct16"):
        keys = W.make_keys(kind, 5, T)
        out, _ = _run(emu, L, 5, 4, keys, T)
        assert (out == np.sort(keys)).all()
    # the blocked layout through phase 9, two layouts for phase 10 and three
    # for phase 11 (as kind 0), two per longer phase, the 16-byte store layout
    assert emu.program_groups(L, 5, 4) == 1 + 2 + (3 if L >= 11 else 0) + \
        2 * max(0, L - 11) + 1


def test_half_tile_sort_program(emu):
    """The half-size scalar-I/O sort with lane steps (2^13 keys, 16 per
    thread, kind 6) that the big-segment tile sort runs on a segment's last
    tile when at most half of it holds keys: sorted, full and partial, at
    most 2-way LDS bank conflicts."""
    T = 1 << 13
    for valid in (T, T - 3, T // 2 + 1, 100, 1):
        keys = W.uniform_i32(valid + 13, T)
        out, steps = _run(emu, 13, 4, 6, keys, valid)
        assert steps == 13 * 14 // 2
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()
    assert emu.worst_bank_conflict_lanes(13, 4, 6, 32, 32) <= 2


@pytest.mark.parametrize("L", [11, 13])
def test_tile_sort_partial(emu, L):
    T = 1 << L
    for valid in (1, 2, 3, 100, T // 2 + 1, T - 1):
        keys = W.uniform_i32(valid, T)
        out, _ = _run(emu, L, 5, 0, keys, valid)
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()


@pytest.mark.parametrize("L", [11, 12, 13, 14, 15])
def test_tile_merge_program(emu, L):
    """The merge tail sorts any tile whose halves at every level were left
    in the state a long-stride pass leaves: here, a bitonic tile (ascending
    then descending) -- a half-cleaner cascade sorts exactly those."""
    T = 1 << L
    for seed in range(3):
        keys = W.uniform_i32(seed + 10, T)
        cut = int(W.uniform_i32(seed + 20, 1)[0]) % T
        bit = np.concatenate([np.sort(keys[:cut]), np.sort(keys[cut:])[::-1]])
        out, steps = _run(emu, L, 5, 1, bit, T)
        assert steps == L
        assert (out == np.sort(keys)).all()


@pytest.mark.parametrize("L,r,kind", [(12, 5, 5), (13, 5, 5), (14, 5, 5), (15, 5, 5), (15, 5, 7),
                                      (12, 4, 7), (13, 4, 7), (14, 4, 7)])
def test_tile_phase_program(emu, L, r, kind):
    """Kinds 5 and 7 (vector and scalar I/O; 4-byte keys at r = 5, 8-byte
    elements at r = 4), all of phase L on a tile whose
    halves are each ascending (as the tile sort of 2^(L-1)-key tiles leaves
    them): the mirror step and L-1 half-cleaners, L steps, tile sorted; for
    partial tiles too (absent keys are the virtual sentinels)."""
    T = 1 << L
    for seed in range(3):
        keys = W.uniform_i32(seed + 40, T)
        two = np.concatenate([np.sort(keys[:T // 2]), np.sort(keys[T // 2:])])
        out, steps = _run(emu, L, r, kind, two, T)
        assert steps == L
        assert (out == np.sort(keys)).all()
    for valid in (T - 1, T // 2 + 5):
        keys = W.uniform_i32(valid, T)
        two = keys.copy()
        two[:T // 2] = np.sort(keys[:T // 2])
        two[T // 2:valid] = np.sort(keys[T // 2:valid])
        out, _ = _run(emu, L, r, kind, two, valid)
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == two[valid:]).all()
    # load layout, the merge layouts of phase L, store layout
    assert emu.program_groups(L, r, kind) == 2 + -(-L // r)


@pytest.mark.parametrize("L", [11, 12, 13, 14, 15])
@pytest.mark.parametrize("kind", [0, 1])
def test_lds_bank_conflicts(emu, L, kind):
    # no half-wave access of any regrouping puts two lanes on one bank
    assert emu.worst_bank_conflict(L, 5, kind, 32) == 1
    assert emu.worst_bank_conflict(L, 5, kind, 64) == 1


@pytest.mark.parametrize("L", list(range(5, 14)))
def test_scalar_io_programs(emu, L):
    """Programs with scalar I/O (used for segments, any alignment): sort and
    merge, full and partial tiles, down to one thread per 32-key tile."""
    T = 1 << L
    for valid in sorted({T, T - 1, T // 2 + 3, 1, 2}):
        if valid < 1:
            continue
        keys = W.uniform_i32(L * 1000 + valid, T)
        out, steps = _run(emu, L, 5, 2, keys, valid)
        assert steps == L * (L + 1) // 2
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()
    keys = W.uniform_i32(L + 77, T)
    cut = T // 3
    bit = np.concatenate([np.sort(keys[:cut]), np.sort(keys[cut:])[::-1]])
    out, steps = _run(emu, L, 5, 3, bit, T)
    assert steps == L and (out == np.sort(keys)).all()
    if L > 5:
        assert emu.worst_bank_conflict(L, 5, 2, 32) == 1
        assert emu.worst_bank_conflict(L, 5, 3, 32) == 1


@pytest.mark.parametrize("L", [11, 12, 13])
def test_wide_programs(emu, L):
    """The programs of the 8-byte tile kernels: 16 elements per thread (r = 4),
    scalar I/O, LDS padded after every 16 words.  Sort and merge, full and
    partial tiles.  The layouts are conflict-free for 8-byte LDS words (16
    lanes per access cycle over 32 two-word banks); the kernels regroup high
    and low words in turn through 4-byte words, where a half-wave meets at
    most 2-way conflicts."""
    T = 1 << L
    for valid in (T, T - 1, T // 2 + 3, 1):
        keys = W.uniform_i32(L * 31 + valid, T)
        out, steps = _run(emu, L, 4, 2, keys, valid)
        assert steps == L * (L + 1) // 2
        assert (out[:valid] == np.sort(keys[:valid])).all()
        assert (out[valid:] == keys[valid:]).all()
    keys = W.uniform_i32(L + 91, T)
    cut = T // 5
    bit = np.concatenate([np.sort(keys[:cut]), np.sort(keys[cut:])[::-1]])
    out, steps = _run(emu, L, 4, 3, bit, T)
    assert steps == L and (out == np.sort(keys)).all()
    for kind in (2, 3):
        assert emu.worst_bank_conflict_lanes(L, 4, kind, 32, 16) == 1
        assert emu.worst_bank_conflict_lanes(L, 4, kind, 32, 32) <= 2


# Every tile program a kernel instantiates: (L, r, kind) -- the single-array
# 4-byte tiles (vector I/O, and the 2^13 scalar-I/O tile), the 8-byte tiles,
# the segmented small-segment programs and big-segment tiles.
INSTANTIATED = sorted({(L, 5, k) for L in range(11, 16) for k in (0, 1, 4)} |
                      {(L, 5, 5) for L in range(12, 16)} | {(15, 5, 7), (13, 4, 6)} |
                      {(L, 4, 7) for L in (12, 13, 14)} |
                      {(13, 5, 6), (13, 5, 3), (14, 5, 6), (14, 5, 3)} |
                      {(L, 4, k) for L in (11, 12, 13) for k in (2, 3)} |
                      {(L, 5, k) for L in range(5, 14) for k in (2, 6)} |
                      {(13, 4, 2), (13, 4, 3)})


@pytest.mark.parametrize("L,r,kind", INSTANTIATED)
def test_in_wave_regroups(emu, L, r, kind):
    """Regroups that the kernels synchronise per wave instead of per
    workgroup must keep every key inside its 64-lane wave: checked against
    every thread and slot of the program; the layout test the kernels use
    finds exactly the regroups the exhaustive check finds."""
    exact = ctypes.c_int()
    got = emu.in_wave_regroups(L, r, kind, ctypes.byref(exact))
    assert got >= 0, "a regroup synchronised per wave moves keys across waves"
    assert got == exact.value
    if L - r <= 6:   # one wave (or less) per tile: every regroup stays inside it
        assert got == emu.program_groups(L, r, kind) - 1
