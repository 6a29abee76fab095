"""The C-ABI library loads and exports every function include/bitonic.h
declares; argument errors come back synchronously; the plan's launch counts
follow the closed forms of sections 3.2-4.2.  No GPU is touched: only calls
that fail argument checks or only count launches are made."""
import ctypes

import pytest

from paper_1506_01446_amd import binding as B


@pytest.fixture(scope="module")
def lib():
    return B.load()


def test_exports_every_declared_symbol(lib):
    names = B.header_functions()
    assert "bitonic_sort_i32" in names and "bitonic_sort_segmented_i32" in names
    missing = [n for n in names if getattr(lib, n, None) is None]
    assert not missing, missing


def test_status_strings(lib):
    for code in B.STATUS:
        assert B.bitonic_status_string(code)
    assert B.bitonic_status_string(12345) == "unknown status"
    assert "gfx950" in B.bitonic_version()


def test_argument_errors_are_synchronous(lib):
    assert lib.bitonic_sort_i32(None, -1, 1, None) == -1
    assert lib.bitonic_sort_i32(None, 5, 1, None) == -1
    assert lib.bitonic_sort_i32(None, 2**31 + 1, 1, None) == -4
    assert lib.bitonic_sort_i32(None, 0, 1, None) == 0
    assert lib.bitonic_sort_i32(None, 1, 0, None) == 0
    bad = B.bitonic_plan(9, 0, 0, 0)
    assert lib.bitonic_sort_plan_i32(None, 0, 1, ctypes.byref(bad), None) == -1
    bad = B.bitonic_plan(3, 17, 0, 0)
    assert lib.bitonic_sort_plan_i32(None, 0, 1, ctypes.byref(bad), None) == -1
    bad = B.bitonic_plan(3, 13, 11, 0)
    assert lib.bitonic_sort_plan_i32(None, 0, 1, ctypes.byref(bad), None) == -1
    bad = B.bitonic_plan(3, 13, 4, 17)
    assert lib.bitonic_sort_plan_i32(None, 0, 1, ctypes.byref(bad), None) == -1
    assert lib.bitonic_network_phases_i32(None, 4, 1, 0, None, None) == -1
    assert lib.bitonic_sort_segmented_i32(None, None, -1, 1, None) == -1
    assert lib.bitonic_sort_segmented_i32(None, None, 0, 1, None) == 0
    assert lib.bitonic_sort_segmented_i32(None, None, 3, 1, None) == -1
    assert lib.bitonic_set_tuning_value(b"seg_fuse", 0) == -1
    assert lib.bitonic_set_tuning_value(b"seg_fuse", 6) == -1
    assert lib.bitonic_sort_segmented_bounded_i32(None, None, 3, -1, 1, None) == -1
    assert lib.bitonic_keygen_i32(None, -1, 0, 0, None) == -1
    assert lib.bitonic_set_tuning(99, 0, 0) == -1
    assert lib.bitonic_set_tuning(0, 11, 0) == -1
    assert lib.bitonic_set_tuning(0, 0, 99) == -1
    assert lib.bitonic_set_tuning(0, 0, -2) == -1
    assert lib.bitonic_load_tuning(b"/nonexistent/tuning.txt") == -1


def test_wide_argument_errors_are_synchronous(lib):
    """8-byte keys and pairs: bad key types, sizes, pointers and plans are
    rejected before anything is enqueued (no pointer here is dereferenced)."""
    I64, F64, I32, F32 = 3, 5, 0, 2
    assert lib.bitonic_sort_keys64(None, -1, I64, 1, None) == -1
    assert lib.bitonic_sort_keys64(None, 5, I64, 1, None) == -1
    assert lib.bitonic_sort_keys64(None, 2**31 + 1, I64, 1, None) == -4
    assert lib.bitonic_sort_keys64(None, 0, I64, 1, None) == 0
    assert lib.bitonic_sort_keys64(None, 1, F64, 0, None) == 0
    assert lib.bitonic_sort_keys64(None, 0, I32, 1, None) == -1     # 4-byte type
    assert lib.bitonic_sort_keys64(None, 0, 6, 1, None) == -1
    assert lib.bitonic_sort_keys64(4, 8, I64, 1, None) == -1        # not 8-byte aligned
    assert lib.bitonic_sort_pairs(None, None, 0, I32, 1, None) == 0
    assert lib.bitonic_sort_pairs(None, None, 1, F32, 1, None) == 0
    assert lib.bitonic_sort_pairs(None, None, 2, I32, 1, None) == -1
    assert lib.bitonic_sort_pairs(None, None, -1, I32, 1, None) == -1
    assert lib.bitonic_sort_pairs(None, None, 0, I64, 1, None) == -1  # 8-byte type
    assert lib.bitonic_sort_pairs(4, 6, 8, I32, 1, None) == -1        # values misaligned
    assert lib.bitonic_sort_pairs(2, 8, 8, I32, 1, None) == -1        # keys misaligned
    for bad in (B.bitonic_plan(1, 0, 0, 0), B.bitonic_plan(3, 14, 0, 0),
                B.bitonic_plan(3, 10, 0, 0), B.bitonic_plan(3, 12, 9, 0)):
        assert lib.bitonic_sort_wide_plan(None, None, 0, I64, 1, ctypes.byref(bad), None) == -1
        assert lib.bitonic_wide_plan_passes(2**20, ctypes.byref(bad)) == -1
    assert lib.bitonic_sort_segmented_pairs(None, None, None, 0, 0, I32, 1, None) == 0
    assert lib.bitonic_sort_segmented_pairs(None, None, None, -1, 0, I32, 1, None) == -1
    assert lib.bitonic_sort_segmented_pairs(4, None, 8, 3, 0, I32, 1, None) == -1   # no values
    assert lib.bitonic_sort_segmented_pairs(4, 6, 8, 3, 0, I32, 1, None) == -1      # misaligned
    assert lib.bitonic_sort_segmented_pairs(4, 8, 8, 3, 0, I64, 1, None) == -1      # 8-byte key
    assert lib.bitonic_sort_segmented_keys(4, 8, 3, 0, I64, 1, None) == -1          # misaligned
    assert lib.bitonic_sort_segmented_keys(8, 8, 3, 0, 6, 1, None) == -1            # no such type
    assert lib.bitonic_sort_segmented_pairs(4, 8, 8, 3, -1, I32, 1, None) == -1
    assert lib.bitonic_set_tuning_value(b"wide_tile_log2", 14) == -1
    assert lib.bitonic_set_tuning_value(b"wide_fuse", 0) == -1


def _closed_form_optimized(k, t, f, phase=True, ragged=False):
    """Launches of the optimized plan on n = 2^k (or, `ragged`, a size that
    pads to 2^k): the tile sort, then per phase p > t its ceil((p - t) / f)
    passes and one merge; passes of more than eight steps (columns split
    over lanes) only up to phase 30, above it at most eight steps (seven
    for a ragged size); with `phase` (16-byte aligned keys, t <= 14) phase
    t + 1 is one launch."""
    if k <= 1:
        return k
    if k <= t:
        return 1
    cap = 7 if ragged else 8
    return 1 + sum(-(-(p - t) // (f if f <= cap or p <= 30 else cap)) + 1
                   for p in range(t + 1, k + 1)) - (1 if phase and t <= 14 else 0)


@pytest.mark.parametrize("t", [11, 12, 13, 14, 15])
@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 6, 7, 8, 9, 10])
def test_optimized_pass_count(lib, t, f):
    for k in range(1, 32):
        n = 2**k
        got = B.bitonic_plan_passes(n, ("optimized", t, f))
        assert got == _closed_form_optimized(k, t, f), (k, t, f)
        # a non-power-of-two n makes the launches of its padded size, its
        # passes of eight to ten steps as lane passes up to phase 30
        if k >= 2:
            assert B.bitonic_plan_passes(n - 1, ("optimized", t, f)) == \
                _closed_form_optimized(k, t, f, ragged=True), (k, t, f)


def _closed_form_wide(k, t, f, phase, pow2=True):
    """Launches of an 8-byte sort on n = 2^k (or a ragged n of that padded
    size): as the 4-byte plan, with passes of more than six steps (lane
    passes) only for powers of two and up to phase 29."""
    if k <= 1:
        return k
    if k <= t:
        return 1
    return 1 + sum(-(-(p - t) // (f if f <= 6 or (pow2 and p <= 29) else 6)) + 1
                   for p in range(t + 1, k + 1)) - (1 if phase else 0)


@pytest.mark.parametrize("t", [11, 12, 13])
@pytest.mark.parametrize("f", [1, 2, 3, 4, 5, 6, 7, 8])
def test_wide_pass_count(lib, t, f):
    """The 8-byte sorts run the optimized plan's schedule (section 4: one
    tile sort, then per phase beyond the tile its fused passes and a merge)."""
    phase = B.bitonic_get_tuning_value("phase_merge") == 1
    for k in range(1, 32):
        got = B.bitonic_wide_plan_passes(2**k, ("optimized", t, f))
        assert got == _closed_form_wide(k, t, f, phase), (k, t, f)
        if k >= 2:
            assert B.bitonic_wide_plan_passes(2**k - 1, ("optimized", t, f)) == \
                _closed_form_wide(k, t, f, phase, pow2=False), (k, t, f)


def test_basic_plan_is_one_launch_per_round(lib):
    # section 3.3: N = 2^k keys need k(k+1)/2 rounds, one kernel each
    for k in range(1, 32):
        assert B.bitonic_plan_passes(2**k, "basic") == k * (k + 1) // 2


def test_semi_plan_counts(lib):
    for t in (8, 12):
        for k in range(1, 28):
            L = min(k, t)
            want = 1 + sum((p - L) + 1 for p in range(L + 1, k + 1))
            assert B.bitonic_plan_passes(2**k, ("semi", t)) == want


def test_headline_pass_count(lib):
    # n = 2^24 with 2^13-key tiles and up to 4 fused steps per HBM pass
    assert B.bitonic_plan_passes(2**24, ("optimized", 13, 4)) == 32  # phase 14 in one launch
    # default: 2^14 tiles, up to 10 fused steps (one pass per phase), phase
    # 15 as one launch
    assert B.bitonic_plan_passes(2**24) == 20
    assert B.bitonic_plan_passes(0) == 0 and B.bitonic_plan_passes(1) == 0
    assert B.bitonic_plan_passes(-1) == -1


def test_default_tile_by_n(lib):
    """The library's tile choice (measured: smaller tiles below 2^21 keys)."""
    saved = B.bitonic_get_tuning_value("tile_log2")
    B.bitonic_set_tuning_value("tile_log2", 0)
    try:
        for k, t in ((2, 12), (16, 12), (17, 13), (20, 13), (21, 14), (24, 14), (31, 14)):
            assert B.bitonic_plan_tile_log2(2**k) == t, k
            assert B.bitonic_plan_tile_log2(2**k - 1 if k > 1 else 2) == t, k
        assert B.bitonic_plan_tile_log2(2**24, ("optimized", 11, 4)) == 11
        assert B.bitonic_plan_tile_log2(2**24, ("semi",)) == 12
        assert B.bitonic_plan_tile_log2(2**24, ("basic",)) == 0
        assert B.bitonic_plan_passes(2**16) == _closed_form_optimized(16, 12, 8)
        B.bitonic_set_tuning_value("tile_log2", 13)
        assert B.bitonic_plan_tile_log2(2**24) == 13 and B.bitonic_plan_tile_log2(2**12) == 13
        B.bitonic_set_tuning_value("tile_log2", 0)
        assert B.bitonic_plan_tile_log2(2**24) == 14
    finally:
        B.bitonic_set_tuning_value("tile_log2", saved)


def test_tuning_values_round_trip(lib, tmp_path):
    from paper_1506_01446_amd import autotune
    saved = {k: B.bitonic_get_tuning_value(k) for k in
             ("tile_log2", "fuse", "merge_blocks_per_cu", "seg_blocks_per_cu",
              "seg_pass_blocks_per_cu")}
    try:
        p = tmp_path / "tuning.txt"
        autotune.write_tuning(str(p), {"tile_log2": 12, "fuse": 3, "merge_blocks_per_cu": 4,
                                       "seg_blocks_per_cu": 2, "seg_pass_blocks_per_cu": 12})
        B.bitonic_load_tuning(str(p))
        assert B.bitonic_get_tuning_value("tile_log2") == 12
        assert B.bitonic_get_tuning_value("fuse") == 3
        assert B.bitonic_get_tuning_value("merge_blocks_per_cu") == 4
        assert B.bitonic_get_tuning_value("seg_blocks_per_cu") == 2
        assert B.bitonic_get_tuning_value("seg_pass_blocks_per_cu") == 12
        # the default plan follows the tuning
        assert B.bitonic_plan_passes(2**24) == _closed_form_optimized(24, 12, 3)
        with pytest.raises(B.BitonicError):
            B.bitonic_set_tuning_value("no_such_knob", 1)
        with pytest.raises(B.BitonicError):
            B.bitonic_set_tuning_value("seg_blocks_per_cu", 0)
        B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", 16)
        assert B.bitonic_get_tuning_value("seg_pass_blocks_per_cu") == 16
        for bad in (0, 33):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", bad)
    finally:
        for k, v in saved.items():
            B.bitonic_set_tuning_value(k, v)
    assert B.bitonic_get_tuning_value("merge_blocks_per_cu") == saved["merge_blocks_per_cu"]


def test_graph_capture_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.bitonic_graph_capture_sort_i32(None, None, 0, 1, None) == -1
    assert lib.bitonic_graph_capture_sort_i32(ctypes.byref(h), None, 5, 1, None) == -1
    assert lib.bitonic_graph_capture_segmented_i32(ctypes.byref(h), None, None, 3, 0, 1) == -1
    assert lib.bitonic_graph_launch(None, None) == -1
    assert lib.bitonic_graph_destroy(None) == 0


def test_bench_traffic_lookup(monkeypatch):
    import bench
    got = bench.committed_traffic("tile_merge", 1 << 24)
    if got is not None:   # the committed counters match the current kernel sources
        assert abs(got / (8 * (1 << 24)) - 1) < 0.05
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0000000000000000")
    assert bench.committed_traffic("tile_merge", 1 << 24) is None
    assert bench.committed_traffic("tile_merge", 12345) is None


def test_bench_kernel_classes():
    import bench
    cases = {
        "tile_kernel<14, 5, 4, 0>": "tile_sort",
        "tile_loop_kernel<14, 5, 1, 0>": "tile_merge",
        "tile_loop_kernel<15, 5, 5, 0>": "tile_phase",
        "global_pass_kernel<3, true, false>": "global_pass_f3",
        "global_pass_kernel<3, true, true>": None,
        "column_pass_kernel<7, true, false, Keys32, false>": "global_pass_f7",
        "column_lanes_pass_kernel<8, 2, true>": "global_pass_f10",
        "column_waves_pass_kernel<7, true>": "global_pass_f9",
        "keygen_kernel": None,
    }
    for name, cls in cases.items():
        assert bench.kernel_class(name) == cls, name


def _ceil_log2(n):
    return max(0, (n - 1).bit_length())


# n = 2^k, 2^k - 1 (k = 1..31) and the first size past 2^30 that is not a
# power of two, where phase 31's mirror step can run as a pass on its own
SHAPE_SIZES = sorted({2**k for k in range(1, 32)} | {2**k - 1 for k in range(2, 32)}
                     | {2**30 + 2**20})


def _check_shapes(shapes, n, elem_bytes, wide=False):
    k = _ceil_log2(n)
    for s in shapes:
        assert s["elem_bytes"] == elem_bytes
        # every byte offset a kernel adds to a row (pass, step) or tile start
        # fits its width: rows of 2^q elements span 2^q * elem_bytes bytes
        assert (1 << s["q"]) * s["elem_bytes"] <= 2 ** s["offset_bits"], (n, s)
        if s["kind"] in ("global_pass", "step"):
            assert 1 <= s["fuse"] and s["q"] + s["fuse"] <= k <= 31, (n, s)
        if wide and s["kind"] == "global_pass" and s["fuse"] > 6:
            # an 8-byte lane pass: whole blocks, lane offsets of 8-byte units
            assert n == 1 << k and (1 << (s["q"] + s["fuse"])) * 8 <= 2 ** 32, (n, s)
        if s["kind"] == "global_pass" and s["fuse"] > 8:
            # a lane pass: its lane byte offsets span the block (the last
            # block of a ragged size padded virtually)
            assert elem_bytes == 4 and s["q"] + s["fuse"] <= 30, (n, s)
            assert (1 << (s["q"] + s["fuse"])) * 4 <= 2 ** s["offset_bits"], (n, s)
        if s["kind"] == "global_pass" and s["fuse"] > 7 and n != 1 << k:
            # a ragged size's eight-step passes are lane passes too
            assert s["q"] + s["fuse"] <= 30, (n, s)


@pytest.mark.parametrize("layout", ["keys32", "keys32_unaligned"])
def test_plan_shapes_4byte(lib, layout):
    """Every launch shape the 4-byte planner can emit for n <= 2^31, under
    every optimized plan and the Basic and Semi plans, keeps its byte
    offsets within their width; the shapes are the plan's launches."""
    plans = [None, "basic", ("semi", 8), ("semi", 13)] + \
        [("optimized", t, f) for t in (11, 12, 13, 14, 15) for f in range(1, 11)]
    for plan in plans:
        for n in SHAPE_SIZES:
            sh = B.bitonic_plan_shapes(n, layout, plan)
            if layout == "keys32":
                assert len(sh) == B.bitonic_plan_passes(n, plan), (plan, n)
            _check_shapes(sh, n, 4)


@pytest.mark.parametrize("layout,unit", [("keys64", 8), ("pairs", 4)])
def test_plan_shapes_8byte(lib, layout, unit):
    """The 8-byte planner under every accepted plan (tiles 2^11..2^13, 1..8
    fused steps, 7 and 8 as lane passes) for n <= 2^31: every pass keeps its
    byte offsets within their width.  One-step passes of phase 31 over
    8-byte keys span 2^33 bytes per row, so they must take 64-bit offsets."""
    wide_q30 = 0
    for t in (11, 12, 13):
        for f in range(1, 9):
            plan = ("optimized", t, f)
            for n in SHAPE_SIZES:
                sh = B.bitonic_plan_shapes(n, layout, plan)
                assert len(sh) == B.bitonic_wide_plan_passes(n, plan), (plan, n)
                _check_shapes(sh, n, unit, wide=True)
                wide_q30 += sum(1 for s in sh if s["kind"] == "global_pass" and s["q"] == 30)
    assert wide_q30 > 0   # the case that needs 64-bit offsets is reached
    sh = B.bitonic_plan_shapes(2**30 + 2**20, layout, ("optimized", 13, 1))
    q30 = [s for s in sh if s["kind"] == "global_pass" and s["q"] == 30]
    assert q30 and all(s["offset_bits"] == (64 if unit == 8 else 32) for s in q30)


@pytest.mark.parametrize("layout,unit", [("seg_keys32", 4), ("seg_pairs", 4),
                                         ("seg_keys64", 8)])
def test_plan_shapes_segmented(lib, layout, unit):
    """The segmented planner, for a longest segment of 1..2^31 elements:
    prep, the small-segment kernel, and for segments past 2^13 elements the
    tile sort and per phase its passes (at most "seg_fuse" steps each) and
    merge; phase T + 1 in one launch (a tile merge with the mirror step, on
    2^(T+1)-element units), with "phase_merge" on."""
    T = 14 if layout == "seg_keys32" else 13   # big-segment tile: 2^14 keys, 2^13 8-byte elements
    phase = B.bitonic_get_tuning_value("phase_merge") == 1
    for k in range(0, 32):
        n = 2**k
        sh = B.bitonic_plan_shapes(n, layout)
        assert [s["kind"] for s in sh[:2]] == ["seg_prep", "seg_small"]
        _check_shapes(sh, n, unit)
        if k <= 13:
            assert len(sh) == 2
            continue
        assert sh[2]["kind"] == "tile_sort" and sh[2]["q"] == T
        merges = [s for s in sh if s["kind"] == "tile_merge"]
        passes = [s for s in sh if s["kind"] == "global_pass"]
        assert len(merges) == max(0, k - T)
        if phase and k > T:
            assert merges[0]["mirror"] == 1 and merges[0]["q"] == T + 1 and sh[3] == merges[0]
        assert all(s["fuse"] <= B.bitonic_get_tuning_value("seg_fuse") for s in passes)
        assert all(s["q"] >= T for s in passes)
        # every phase p > T performs steps on bits p-1 .. T exactly once (the
        # tile phase those of phase T + 1)
        done = 1 if phase and k > T else 0
        assert sum(s["fuse"] for s in passes) + done == sum(p - T for p in range(T + 1, k + 1))


def test_noalloc_argument_errors(lib):
    """The allocation-free segmented sort checks its sizes before it takes
    its scratch array's address (no device is touched here)."""
    assert lib.bitonic_sort_segmented_noalloc_i32(None, None, 0, 0, 1, None) == 0
    assert lib.bitonic_sort_segmented_noalloc_i32(None, None, -1, 8, 1, None) == -1
    assert lib.bitonic_sort_segmented_noalloc_i32(None, None, 2**18, 8, 1, None) == -4
    assert lib.bitonic_sort_segmented_noalloc_i32(None, None, 3, 2**31 + 1, 1, None) == -4
    assert lib.bitonic_sort_segmented_noalloc_i32(None, None, 3, 0, 1, None) == -1
    assert lib.bitonic_sort_segmented_noalloc_i32(None, 8, 3, 8, 1, None) == -1
    assert lib.bitonic_sort_segmented_noalloc_i32(6, 8, 3, 8, 1, None) == -1   # misaligned


def test_segmented_default_bound_arguments(lib):
    assert lib.bitonic_segmented_default_bound(None, 4) == -1
    assert lib.bitonic_segmented_default_bound(64, 2) == -1


def test_bucket_tuning(lib, tmp_path):
    """Per-size-bucket plan entries ("name@k"): they set the plan of that
    size only, take precedence over the global values, and load from a
    tuning file with comments."""
    k = 22
    try:
        B.bitonic_set_tuning_value(f"tile_log2@{k}", 13)
        B.bitonic_set_tuning_value(f"fuse@{k}", 5)
        assert B.bitonic_get_tuning_value(f"tile_log2@{k}") == 13
        assert B.bitonic_plan_tile_log2(2**k) == 13
        assert B.bitonic_plan_tile_log2(2**k - 5) == 13
        assert B.bitonic_plan_tile_log2(2**(k + 1)) == 14          # other buckets untouched
        assert B.bitonic_plan_passes(2**k) == _closed_form_optimized(k, 13, 5)
        assert B.bitonic_plan_passes(2**k, ("optimized", 14, 8)) == _closed_form_optimized(k, 14, 8)
        B.bitonic_set_tuning_value(f"lane_pass@{k}", 9)
        assert B.bitonic_get_tuning_value(f"lane_pass@{k}") == 9
        with pytest.raises(B.BitonicError):
            B.bitonic_set_tuning_value(f"lane_pass@{k}", 5)
        B.bitonic_set_tuning_value(f"lane_pass@{k}", 0)
        for bad in ("tile_log2@32", "fuse@-1", "nonsense@3", "tile_log2@x"):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value(bad, 13)
        with pytest.raises(B.BitonicError):
            B.bitonic_set_tuning_value(f"fuse@{k}", 11)
        p = tmp_path / "t.txt"
        p.write_text(f"# tuned table\nmerge_blocks_per_cu@{k} 4   # four per CU\n\nfuse@{k} 6\n")
        B.bitonic_load_tuning(str(p))
        assert B.bitonic_get_tuning_value(f"merge_blocks_per_cu@{k}") == 4
        assert B.bitonic_get_tuning_value(f"fuse@{k}") == 6
        p.write_text("fuse@3 6 7\n")
        with pytest.raises(B.BitonicError):
            B.bitonic_load_tuning(str(p))
    finally:
        for name in ("tile_log2", "fuse", "merge_blocks_per_cu"):
            B.bitonic_set_tuning_value(f"{name}@{k}", 0)
    assert B.bitonic_plan_tile_log2(2**k) == 14


def test_validation_switch(lib):
    """Offsets validation is a switch ("validate", 0 or 1; off unless
    BITONIC_VALIDATE=1 is set); its error query needs an output pointer."""
    import os
    saved = B.bitonic_get_tuning_value("validate")
    assert saved == (1 if os.environ.get("BITONIC_VALIDATE") == "1" else 0)
    for bad in (-1, 2):
        with pytest.raises(B.BitonicError):
            B.bitonic_set_tuning_value("validate", bad)
    B.bitonic_set_tuning_value("validate", 1)
    assert B.bitonic_get_tuning_value("validate") == 1
    B.bitonic_set_tuning_value("validate", saved)
    assert lib.bitonic_validation_error(None) == -1


def test_autotune_summary(lib, tmp_path):
    """The autotuner's summary keeps the five fastest plans per bucket, the
    winner, and every segmented and 8-byte timing."""
    import json
    from paper_1506_01446_amd import autotune
    rows = [{"bucket": 20, "tile_log2": t, "fuse": 8, "merge_blocks_per_cu": -1, "ms": 1.0 + t}
            for t in range(12, 19)]
    rows.append({"bucket": 20, "best": {"tile_log2": 12, "ms": 13.0, "default_ms": 14.0}})
    rows.append({"bucket": 20, "sort_tile_log2": 15, "ms": 30.0})
    rows.append({"seg_blocks_per_cu": 4, "ms": 0.5})
    p = tmp_path / "summary.txt"
    autotune.write_summary(str(p), rows, "cmd")
    body = [json.loads(ln) for ln in p.read_text().splitlines() if ln.startswith("{")]
    assert [r["tile_log2"] for r in body if "tile_log2" in r][:5] == [12, 13, 14, 15, 16]
    assert any("best" in r for r in body) and body[-1] == {"seg_blocks_per_cu": 4, "ms": 0.5}
    assert {"bucket": 20, "sort_tile_log2": 15, "ms": 30.0} in body   # kept though slow
    assert "slowest 30.0 ms" in p.read_text()
    # a bucket's sort-tile entry goes into the table and loads back
    t = tmp_path / "table.txt"
    autotune.write_tuning(str(t), {"buckets": {24: {"tile_log2": 14, "fuse": 10,
                                                    "merge_blocks_per_cu": 2, "ms": 1.0,
                                                    "default_ms": 1.0, "sort_tile_log2": 15}}})
    lines = t.read_text().splitlines()
    # the bucket's plan goes with its tile-sort entry, though it does not
    # beat the built-in plan by itself
    assert "sort_tile_log2@24 15" in lines and "tile_log2@24 14" in lines
    saved = B.bitonic_get_tuning_value("sort_tile_log2@24")
    try:
        B.bitonic_load_tuning(str(t))
        assert B.bitonic_get_tuning_value("sort_tile_log2@24") == 15
    finally:
        B.bitonic_set_tuning_value("sort_tile_log2@24", saved)


def test_lane_pass_modes(lib):
    """Passes of nine and ten steps exist only with lane passes on, for
    arrays on a 16-byte boundary (a ragged size's lane passes are all
    column-over-lanes ones, whatever the mode); off, or for other arrays, a
    pass takes at most eight steps (seven for ragged sizes)."""
    saved = B.bitonic_get_tuning_value("lane_pass")
    try:
        for bad in (1, 6, 10, -1):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("lane_pass", bad)
        for mode in (7, 8, 9):
            B.bitonic_set_tuning_value("lane_pass", mode)
            assert B.bitonic_get_tuning_value("lane_pass") == mode
            for f in (9, 10):
                assert B.bitonic_plan_passes(2**24, ("optimized", 14, f)) == \
                    _closed_form_optimized(24, 14, f)
                fuses = [s["fuse"] for s in B.bitonic_plan_shapes(2**24, "keys32", ("optimized", 14, f))
                         if s["kind"] == "global_pass"]
                assert max(fuses) == f
                assert max(s["fuse"] for s in B.bitonic_plan_shapes(
                    2**24, "keys32_unaligned", ("optimized", 14, f))
                    if s["kind"] == "global_pass") == 8
                assert B.bitonic_plan_passes(2**24 - 1, ("optimized", 14, f)) == \
                    _closed_form_optimized(24, 14, f, ragged=True)
                assert max(s["fuse"] for s in B.bitonic_plan_shapes(
                    10**7, "keys32", ("optimized", 14, f)) if s["kind"] == "global_pass") == f
        B.bitonic_set_tuning_value("lane_pass", 0)
        assert B.bitonic_plan_passes(2**24 - 1, ("optimized", 14, 10)) == \
            _closed_form_optimized(24, 14, 7, ragged=True)
        assert B.bitonic_plan_passes(2**24, ("optimized", 14, 10)) == \
            _closed_form_optimized(24, 14, 8)
    finally:
        B.bitonic_set_tuning_value("lane_pass", saved)


def _closed_form_sort_tile(k, t, f, s, phase=True):
    """Launches of the optimized plan on n = 2^k whose tile sort takes 2^s-key
    tiles (s >= t): phases 1..s in one launch, then per phase p > s its
    ceil((p - t) / f) passes down to bit t and a merge of 2^t-key tiles;
    phase s + 1 in one launch when s <= 14."""
    if k <= 1:
        return k
    if k <= s:
        return 1
    per = [-(-(p - t) // (f if f <= 8 or p <= 30 else 8)) + 1 for p in range(s + 1, k + 1)]
    if phase and s <= 14:
        per[0] = 1
    return 1 + sum(per)


def test_sort_tile(lib):
    """A tile-sort tile larger than the merge tile ("sort_tile_log2"): for
    n a power of two the tile sort takes phases 1..s, every later phase's
    passes cover its strides from 2^(p-1) down to the merge tile 2^t, each
    once, and its merge the rest; other sizes, and arrays off a 16-byte
    boundary, keep the plan's tile."""
    saved = B.bitonic_get_tuning_value("sort_tile_log2")
    saved24 = B.bitonic_get_tuning_value("sort_tile_log2@24")
    try:
        for bad in (-1, 1, 10, 16):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("sort_tile_log2", bad)
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("sort_tile_log2@24", bad)
        for s in (12, 13, 14, 15):
            B.bitonic_set_tuning_value("sort_tile_log2", s)
            assert B.bitonic_get_tuning_value("sort_tile_log2") == s
            for t in (11, 12, 13, 14, 15):
                for f in (2, 7, 10):
                    plan = ("optimized", t, f)
                    for k in range(1, 32):
                        assert B.bitonic_plan_passes(2**k, plan) == \
                            _closed_form_sort_tile(k, t, f, max(s, t)), (s, t, f, k)
                    for n in (2**24, 2**24 - 1, 10**7, 2**s + 5, 2**31, 2**(s - 1)):
                        sh = B.bitonic_plan_shapes(n, "keys32", plan)
                        k = _ceil_log2(n)
                        # a larger tile sort only for powers of two
                        ls = max(s, t) if n & (n - 1) == 0 else t
                        assert sh[0]["kind"] == "tile_sort" and sh[0]["q"] == min(ls, k)
                        i, p = 1, ls + 1
                        while i < len(sh):   # one phase: passes, then its merge
                            if p == ls + 1 and ls <= 14:
                                assert sh[i]["kind"] == "tile_merge" and sh[i]["q"] == p
                                i, p = i + 1, p + 1
                                continue
                            top = p - 1
                            while sh[i]["kind"] == "global_pass":
                                assert sh[i]["q"] + sh[i]["fuse"] - 1 == top
                                assert sh[i]["mirror"] == (1 if top == p - 1 else 0)
                                top = sh[i]["q"] - 1
                                i += 1
                            assert top == t - 1, (s, t, f, n, p)
                            assert sh[i]["kind"] == "tile_merge" and sh[i]["q"] == t
                            i, p = i + 1, p + 1
                        assert p == max(k, ls) + 1, (s, t, f, n)
                        _check_shapes(sh, n, 4)
                    un = B.bitonic_plan_shapes(2**24, "keys32_unaligned", plan)
                    assert un[0]["q"] == 13 and all(x["q"] == 13 for x in un
                                                    if x["kind"] == "tile_merge")
        B.bitonic_set_tuning_value("sort_tile_log2", 0)
        assert B.bitonic_plan_passes(2**24, ("optimized", 14, 10)) == \
            _closed_form_optimized(24, 14, 10)
        # a size-bucket entry applies to its bucket only
        B.bitonic_set_tuning_value("sort_tile_log2@24", 15)
        assert B.bitonic_get_tuning_value("sort_tile_log2@24") == 15
        assert B.bitonic_plan_passes(2**24, ("optimized", 14, 10)) == \
            _closed_form_sort_tile(24, 14, 10, 15)
        assert B.bitonic_plan_passes(2**23, ("optimized", 14, 10)) == \
            _closed_form_optimized(23, 14, 10)
    finally:
        B.bitonic_set_tuning_value("sort_tile_log2", saved)
        B.bitonic_set_tuning_value("sort_tile_log2@24", saved24)


def test_phase_merge_switch(lib):
    """Phase t + 1 as one tile-phase launch (a tile merge whose first step
    is the mirror step, on 2^(t+1)-key tiles) for aligned arrays with
    t <= 14; off, a one-step pass and a merge."""
    saved = B.bitonic_get_tuning_value("phase_merge")
    try:
        for bad in (-1, 2):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("phase_merge", bad)
        pb = B.bitonic_get_tuning_value("phase_blocks_per_cu")
        for bad in (-2, 17):
            with pytest.raises(B.BitonicError):
                B.bitonic_set_tuning_value("phase_blocks_per_cu", bad)
        for ok in (-1, 0, 4):
            B.bitonic_set_tuning_value("phase_blocks_per_cu", ok)
            assert B.bitonic_get_tuning_value("phase_blocks_per_cu") == ok
        B.bitonic_set_tuning_value("phase_blocks_per_cu", pb)
        for on in (0, 1):
            B.bitonic_set_tuning_value("phase_merge", on)
            for t in (11, 12, 13, 14, 15):
                for k in (t, t + 1, t + 2, 24):
                    plan = ("optimized", t, 8)
                    assert B.bitonic_plan_passes(2**k, plan) == \
                        _closed_form_optimized(k, t, 8, bool(on)), (on, t, k)
                    sh = B.bitonic_plan_shapes(2**k, "keys32", plan)
                    ph = [s for s in sh if s["kind"] == "tile_merge" and s["mirror"]]
                    assert len(ph) == (1 if on and t <= 14 and k > t else 0)
                    if ph:
                        assert ph[0]["q"] == t + 1 and sh[1] == ph[0]
                    # an array off a 16-byte boundary keeps pass and merge
                    assert not any(s["kind"] == "tile_merge" and s["mirror"] for s in
                                   B.bitonic_plan_shapes(2**k, "keys32_unaligned", plan))
    finally:
        B.bitonic_set_tuning_value("phase_merge", saved)
