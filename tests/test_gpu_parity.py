"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

Keys-only sorting has a unique answer, so every comparison is bit-exact
(tolerance 0).  Inputs come from the seeded generators; expected values come
from the oracle only.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1506_01446_amd import binding as B  # noqa: E402
from paper_1506_01446_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 63, 64, 65, 127, 129, 255, 256,
         257, 1000, 1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193,
         16383, 16385, 32768, 65535, 65536, 65537, 100003, 131075, 262144, 300001]
PLANS = [("basic",), ("semi", 8), ("semi", 12)] + \
        [("optimized", t, f) for t in (11, 12, 13, 14, 15) for f in (1, 2, 3, 4, 5, 6, 7, 8)] + \
        [("optimized", 13, 5, 4), ("optimized", 14, 5, 2), ("optimized", 15, 5, 1),
         ("optimized", 14, 7, 2), ("optimized", 14, 8, 2)]


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()
    print(f"[gpu] {torch.cuda.get_device_name(0)} lib={B.bitonic_version()}", flush=True)


def gpu_sort(keys, ascending=True, plan=None):
    t = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int32)).cuda()
    if plan is None:
        B.bitonic_sort_i32(t, ascending)
    else:
        B.bitonic_sort_plan_i32(t, ascending, plan)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_headline_small_config():
    """n = 2^16 uniform int32, ascending, default plan."""
    keys = W.uniform_i32(W.SEED_BASE + 1, 2**16)
    want = O.sort_i32(keys, True)
    net, _, _ = O.bitonic_i32(keys, True, O.FLIP_VIRTUAL)
    assert (want == net).all()
    for rep in range(5):  # repeated: an LDS race would show as a mismatch
        assert np.array_equal(gpu_sort(keys, True), want), rep


@pytest.mark.parametrize("plan", PLANS, ids=lambda p: "-".join(map(str, p)))
def test_sizes_and_plans(plan):
    for n in SIZES:
        keys = W.uniform_i32(W.SEED_BASE + 7 * n + 3, n)
        for asc in (True, False):
            print(f"[case] plan={plan} n={n} asc={asc}", flush=True)
            got = gpu_sort(keys, asc, plan)
            assert np.array_equal(got, O.sort_i32(keys, asc)), (plan, n, asc)


@pytest.mark.parametrize("kind", W.KINDS)
def test_distributions(kind):
    n = (1 << 20) + 12345
    keys = W.make_keys(kind, W.SEED_BASE + 10, n)
    for asc in (True, False):
        assert np.array_equal(gpu_sort(keys, asc), O.sort_i32(keys, asc)), (kind, asc)


def test_signed_extremes():
    n = 50000
    keys = W.uniform_i32(5, n)
    keys[::7] = 2**31 - 1
    keys[3::11] = -2**31
    keys[5::13] = -1
    for asc in (True, False):
        for plan in (None, ("basic",), ("semi", 12)):
            assert np.array_equal(gpu_sort(keys, asc, plan), O.sort_i32(keys, asc))


@pytest.mark.parametrize("plan", [("optimized", 11, 2, 1), ("optimized", 12, 5, 2),
                                  ("optimized", 14, 5, 1), ("optimized", 15, 5, 1)],
                         ids=lambda p: "-".join(map(str, p)))
def test_merge_loop_kernel(plan):
    """Merges on fewer workgroups than tiles: each block loops over several
    full tiles with its next tile prefetched (an empty prefetch on its last
    iteration) and one block also merges the partial last tile."""
    L, grid = plan[1], torch.cuda.get_device_properties(0).multi_processor_count * plan[3]
    cases = ((grid + 1, 0), (2 * grid, 777), (3 * grid - 5, 1)) if L < 14 else ((grid + 3, 4097),)
    for tiles, tail in cases:
        n = (tiles << L) + tail
        keys = W.uniform_i32(W.SEED_BASE + 31 + n, n)
        for asc in (True, False):
            print(f"[case] plan={plan} n={n} asc={asc}", flush=True)
            assert np.array_equal(gpu_sort(keys, asc, plan), O.sort_i32(keys, asc)), (plan, n, asc)


def test_merge_loop_kernel_float_keys():
    """The last merge decodes float32 keys in the looping kernel."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = ((2 * cus) << 14) + 999
    bits = W.uniform_i32(W.SEED_BASE + 32, n).view(np.uint32).copy()
    bits[: len(TOTAL_ORDER_BITS)] = TOTAL_ORDER_BITS
    old = B.bitonic_get_tuning_value("merge_blocks_per_cu")
    B.bitonic_set_tuning_value("merge_blocks_per_cu", 1)
    try:
        for asc in (True, False):
            t = torch.from_numpy(bits.view(np.int32).copy()).cuda()
            B.bitonic_sort_keys(t, asc, "float32")
            torch.cuda.synchronize()
            want = O.sort_keys(bits.view(np.float32), O.KEY_F32, asc).view(np.int32)
            assert np.array_equal(t.cpu().numpy(), want), asc
    finally:
        B.bitonic_set_tuning_value("merge_blocks_per_cu", old)


@pytest.mark.parametrize("plan", [("optimized", 11, 2), ("optimized", 13, 4),
                                  ("optimized", 14, 5), ("optimized", 15, 3),
                                  ("optimized", 11, 7), ("semi", 9), ("basic",)],
                         ids=lambda p: "-".join(map(str, p)))
def test_per_phase_states(plan):
    """After phase p the GPU state equals the oracle network's state after
    phase p (every aligned 2^p block sorted), for every p."""
    n = (1 << 16) + 4321
    keys = W.uniform_i32(77, n)
    states = {}
    O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                  hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
    for p in sorted(states):
        t = torch.from_numpy(keys.copy()).cuda()
        B.bitonic_network_phases_i32(t, p, True, plan)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), states[p]), (plan, p)


@pytest.mark.parametrize("mode", [8, 7, 9])
def test_lane_passes(mode):
    """Passes of eight to ten steps with each column split over two or four
    lanes (lane passes; with mode 7 eight- and nine-step passes take 2^7
    keys per lane; with mode 9 nine and ten steps spread each column over
    the four waves of a workgroup): every tile size, both directions, at power-of-two sizes
    whose last phases have nine and ten long-stride steps, so that mirror
    and plain lane passes of every width run."""
    saved = B.bitonic_get_tuning_value("lane_pass")
    want = {}
    try:
        B.bitonic_set_tuning_value("lane_pass", mode)
        for t in (11, 12, 13, 14, 15):
            for k in sorted({min(t + 9, 24), min(t + 10, 24)}):
                if k not in want:
                    keys = W.uniform_i32(W.SEED_BASE + 300 + k, 1 << k)
                    want[k] = (keys, O.sort_i32(keys, True))
                keys, w = want[k]
                for f in (8, 9, 10):
                    plan = ("optimized", t, f)
                    assert max(s["fuse"] for s in B.bitonic_plan_shapes(1 << k, "keys32", plan)
                               if s["kind"] == "global_pass") == min(f, k - t)
                    for asc in (True, False):
                        print(f"[case] lane_pass={mode} plan={plan} n=2^{k} asc={asc}", flush=True)
                        got = gpu_sort(keys, asc, plan)
                        assert np.array_equal(got, w if asc else w[::-1]), (mode, plan, k, asc)
    finally:
        B.bitonic_set_tuning_value("lane_pass", saved)


@pytest.mark.parametrize("mode", [7, 9])
def test_lane_passes_ragged(mode):
    """Lane passes over sizes that are not powers of two (the last block of
    each pass padded virtually: keys past n read as the sentinel, never
    stored): eight- to ten-step passes at every tile size, sizes just under
    a power of two, just over one, and in between, both directions."""
    saved = B.bitonic_get_tuning_value("lane_pass")
    want = {}
    try:
        B.bitonic_set_tuning_value("lane_pass", mode)
        for t in (11, 13, 14):
            for n in ((1 << (t + 10)) - 3, (1 << (t + 9)) + 12345, 3 * (1 << (t + 8)) + 7):
                if n > 1 << 24:
                    continue
                if n not in want:
                    keys = W.uniform_i32(W.SEED_BASE + 500 + n % 997, n)
                    want[n] = (keys, O.sort_i32(keys, True))
                keys, w = want[n]
                for f in (8, 9, 10):
                    plan = ("optimized", t, f)
                    sh = B.bitonic_plan_shapes(n, "keys32", plan)
                    assert max(s["fuse"] for s in sh if s["kind"] == "global_pass") == \
                        min(f, (n - 1).bit_length() - t)
                    for asc in (True, False):
                        print(f"[case] ragged lane_pass={mode} plan={plan} n={n} asc={asc}",
                              flush=True)
                        got = gpu_sort(keys, asc, plan)
                        assert np.array_equal(got, w if asc else w[::-1]), (mode, plan, n, asc)
    finally:
        B.bitonic_set_tuning_value("lane_pass", saved)


def test_per_phase_states_ragged_lane_passes():
    """Per-phase states through lane passes over a ragged size: n = 2^21 -
    4099 with 2^11 tiles (phases 19..21 take eight- to ten-step passes whose
    last block straddles n) equals the oracle's virtually padded network."""
    n = (1 << 21) - 4099
    keys = W.uniform_i32(81, n)
    states = {}
    O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                  hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
    for p in range(12, 22):
        print(f"[case] per-phase ragged lane passes p={p}", flush=True)
        t = torch.from_numpy(keys.copy()).cuda()
        B.bitonic_network_phases_i32(t, p, True, ("optimized", 11, 10))
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), states[p]), p


@pytest.mark.parametrize("mode", [7, 9])
@pytest.mark.parametrize("plan", [("optimized", 11, 10), ("optimized", 11, 9)],
                         ids=lambda p: "-".join(map(str, p)))
def test_per_phase_states_lane_passes(plan, mode):
    """Per-phase states through the lane passes: n = 2^21 with 2^11 tiles,
    whose phases 20 and 21 take nine- and ten-step passes."""
    n = 1 << 21
    keys = W.uniform_i32(79, n)
    states = {}
    O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                  hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
    saved = B.bitonic_get_tuning_value("lane_pass")
    try:
        B.bitonic_set_tuning_value("lane_pass", mode)
        for p in range(12, 22):
            print(f"[case] per-phase lane passes plan={plan} mode={mode} p={p}", flush=True)
            t = torch.from_numpy(keys.copy()).cuda()
            B.bitonic_network_phases_i32(t, p, True, plan)
            torch.cuda.synchronize()
            assert np.array_equal(t.cpu().numpy(), states[p]), (plan, p)
    finally:
        B.bitonic_set_tuning_value("lane_pass", saved)


@pytest.mark.parametrize("s", [12, 13, 14, 15])
def test_sort_tile(s):
    """A tile sort of 2^s-key tiles ahead of 2^t-key merges (t < s, tuning
    value "sort_tile_log2", powers of two): every such pair, short and
    ten-step passes, with the tile phase on and off, at powers of two (the
    larger tile sort) and with ragged tails (the plan's tile), looping and
    one-tile merge workgroups, both directions, bit-exact against the
    oracle."""
    saved = B.bitonic_get_tuning_value("sort_tile_log2")
    saved_pm = B.bitonic_get_tuning_value("phase_merge")
    want = {}
    try:
        B.bitonic_set_tuning_value("sort_tile_log2", s)
        for pm in (1, 0):
            B.bitonic_set_tuning_value("phase_merge", pm)
            for t in range(11, s):
                for n in ((1 << s) - 7, 1 << s, 1 << (s + 1), (1 << (s + 2)) + 4099,
                          1 << (s + 4)):
                    if n not in want:
                        keys = W.uniform_i32(W.SEED_BASE + 91 * s + n, n)
                        want[n] = (keys, O.sort_i32(keys, True))
                    keys, w = want[n]
                    for plan in (("optimized", t, 2, -1), ("optimized", t, 10, 2)):
                        pow2 = n & (n - 1) == 0
                        assert B.bitonic_plan_shapes(n, "keys32", plan)[0]["q"] == \
                            min(s if pow2 else t, max(1, (n - 1).bit_length()))
                        for asc in (True, False):
                            print(f"[case] sort_tile={s} phase_merge={pm} plan={plan} n={n} "
                                  f"asc={asc}", flush=True)
                            got = gpu_sort(keys, asc, plan)
                            assert np.array_equal(got, w if asc else w[::-1]), (s, pm, plan, n, asc)
    finally:
        B.bitonic_set_tuning_value("sort_tile_log2", saved)
        B.bitonic_set_tuning_value("phase_merge", saved_pm)


def test_sort_tile_per_phase_states():
    """Per-phase states with 2^15-key tile sorts ahead of 2^11-key merges
    (n = 2^19): the state after every phase from the tile sort's last on
    equals the oracle network's."""
    n = 1 << 19
    keys = W.uniform_i32(83, n)
    states = {}
    O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                  hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
    saved = B.bitonic_get_tuning_value("sort_tile_log2")
    try:
        B.bitonic_set_tuning_value("sort_tile_log2", 15)
        for plan in (("optimized", 11, 3), ("optimized", 14, 10)):
            for p in range(15, 20):
                print(f"[case] per-phase sort_tile=15 plan={plan} p={p}", flush=True)
                t = torch.from_numpy(keys.copy()).cuda()
                B.bitonic_network_phases_i32(t, p, True, plan)
                torch.cuda.synchronize()
                assert np.array_equal(t.cpu().numpy(), states[p]), (plan, p)
    finally:
        B.bitonic_set_tuning_value("sort_tile_log2", saved)


def test_sort_tile_full_size():
    """The 2^24-key bucket with 2^15-key tile sorts (as the plan table may
    choose): n = 2^24, and n = 10,000,000 (virtual padding), which keeps
    the plan's 2^14-key tile sort, both directions, bit-exact against the
    oracle."""
    saved = B.bitonic_get_tuning_value("sort_tile_log2@24")
    try:
        B.bitonic_set_tuning_value("sort_tile_log2@24", 15)
        for n in (1 << 24, 10_000_000):
            keys = W.uniform_i32(W.SEED_BASE + 2 + n, n)
            w = O.sort_i32(keys, True)
            assert B.bitonic_plan_shapes(n, "keys32", None)[0]["q"] == \
                (15 if n == 1 << 24 else B.bitonic_plan_tile_log2(n))
            for asc in (True, False):
                print(f"[case] sort_tile@24=15 n={n} asc={asc}", flush=True)
                got = gpu_sort(keys, asc)
                assert np.array_equal(got, w if asc else w[::-1]), (n, asc)
    finally:
        B.bitonic_set_tuning_value("sort_tile_log2@24", saved)


@pytest.mark.parametrize("t", [11, 12, 13, 14])
def test_phase_merge(t):
    """Phase t + 1 as one launch on 2^(t+1)-key tiles (the tile phase), on
    and off: as the last launch (n = 2^(t+1), keys decoded there, also
    float32 keys), followed by further phases, with a ragged tail, with
    looping workgroups, both directions; and the state after phase t + 1
    equals the oracle network's."""
    saved = B.bitonic_get_tuning_value("phase_merge")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    try:
        for on in (1, 0):
            B.bitonic_set_tuning_value("phase_merge", on)
            for n in (1 << (t + 1), (1 << (t + 1)) - 3, (1 << (t + 3)) + 4099,
                      (3 * cus << (t + 1)) + 5):
                for plan in (("optimized", t, 8, -1), ("optimized", t, 10, 1)):
                    keys = W.uniform_i32(W.SEED_BASE + 57 * t + n, n)
                    for asc in (True, False):
                        print(f"[case] phase_merge={on} plan={plan} n={n} asc={asc}", flush=True)
                        got = gpu_sort(keys, asc, plan)
                        assert np.array_equal(got, O.sort_i32(keys, asc)), (on, plan, n, asc)
            n = 1 << (t + 1)
            bits = W.uniform_i32(W.SEED_BASE + 58, n).view(np.uint32).copy()
            bits[: len(TOTAL_ORDER_BITS)] = TOTAL_ORDER_BITS
            old = B.bitonic_get_tuning_value("tile_log2")
            B.bitonic_set_tuning_value("tile_log2", t)
            try:
                for asc in (True, False):
                    tk = torch.from_numpy(bits.view(np.int32).copy()).cuda()
                    B.bitonic_sort_keys(tk, asc, "float32")
                    torch.cuda.synchronize()
                    want = O.sort_keys(bits.view(np.float32), O.KEY_F32, asc).view(np.int32)
                    assert np.array_equal(tk.cpu().numpy(), want), (on, asc)
            finally:
                B.bitonic_set_tuning_value("tile_log2", old)
            n = (1 << (t + 2)) + 321
            keys = W.uniform_i32(80 + t, n)
            states = {}
            O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                          hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
            for p in (t + 1, t + 2):
                tk = torch.from_numpy(keys.copy()).cuda()
                B.bitonic_network_phases_i32(tk, p, True, ("optimized", t, 8))
                torch.cuda.synchronize()
                assert np.array_equal(tk.cpu().numpy(), states[p]), (on, t, p)
    finally:
        B.bitonic_set_tuning_value("phase_merge", saved)


@pytest.mark.parametrize("shift", [1, 2, 3])
def test_per_phase_states_unaligned(shift):
    """The same on views 1-3 keys past a 16-byte boundary, which take the
    scalar-access plan (2^13-key tiles): phases 1..p for p below the tile
    size must stop at p, not run the whole tile."""
    n = (1 << 15) + 1234
    keys = W.uniform_i32(78 + shift, n)
    states = {}
    O.bitonic_i32(keys, True, O.FLIP_VIRTUAL,
                  hook=lambda p, s, x: states.__setitem__(p, x) if s == p else None)
    buf = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
    for p in sorted(states):
        buf[shift:shift + n] = torch.from_numpy(keys).cuda()
        v = buf[shift:shift + n]
        assert v.data_ptr() % 16 != 0
        B.bitonic_network_phases_i32(v, p, True)
        torch.cuda.synchronize()
        assert np.array_equal(v.cpu().numpy(), states[p]), (shift, p)


def test_guard_bands():
    n = 300001
    keys = W.uniform_i32(9, n)
    canary = np.int32(0x5AFE5AFE)
    buf = torch.full((n + 2048,), int(canary), dtype=torch.int32, device="cuda")
    buf[1024:1024 + n] = torch.from_numpy(keys).cuda()
    for asc in (True, False):
        B.bitonic_sort_i32(buf[1024:1024 + n], asc)
        torch.cuda.synchronize()
        h = buf.cpu().numpy()
        assert (h[:1024] == canary).all() and (h[1024 + n:] == canary).all()
        assert np.array_equal(h[1024:1024 + n], O.sort_i32(keys, asc))


def test_unaligned_pointers():
    """Views that start 4, 8 or 12 bytes past a 16-byte boundary (the
    optimized plan's 16-byte accesses need alignment; such arrays take its
    scalar-access tiles and one-column passes): sorted, and nothing outside
    the view is touched."""
    canary = np.int32(0x5AFE5AFE)
    for n in (1000, 8192, 8193, 70001, (1 << 20) + 3, (1 << 24) - 5):
        keys = W.uniform_i32(W.SEED_BASE + 60 + n, n)
        for shift in ((1, 2, 3) if n < (1 << 24) - 5 else (1,)):
            buf = torch.full((n + 64,), int(canary), dtype=torch.int32, device="cuda")
            buf[shift:shift + n] = torch.from_numpy(keys).cuda()
            for asc, plan in ((True, None), (False, ("optimized", 14, 8))):
                view = buf[shift:shift + n]
                print(f"[case] unaligned n={n} shift={shift} asc={asc} plan={plan}", flush=True)
                if plan is None:
                    B.bitonic_sort_i32(view, asc)
                else:
                    B.bitonic_sort_plan_i32(view, asc, plan)
                torch.cuda.synchronize()
                h = buf.cpu().numpy()
                assert (h[:shift] == canary).all() and (h[shift + n:] == canary).all()
                assert np.array_equal(h[shift:shift + n], O.sort_i32(keys, asc)), (n, shift)
        bits = keys.view(np.uint32)
        for key_type, kt, dt in (("uint32", O.KEY_U32, np.uint32), ("float32", O.KEY_F32, np.float32)):
            buf = torch.full((n + 8,), int(canary), dtype=torch.int32, device="cuda")
            buf[3:3 + n] = torch.from_numpy(keys).cuda()
            B.bitonic_sort_keys(buf[3:3 + n], True, key_type)
            torch.cuda.synchronize()
            h = buf.cpu().numpy()
            assert (h[:3] == canary).all() and (h[3 + n:] == canary).all()
            want = O.sort_keys(bits.view(dt), kt, True).view(np.int32)
            assert np.array_equal(h[3:3 + n], want), key_type


def test_keygen_matches_host_generator():
    for seed, start, n in ((1, 0, 1000), (W.SEED_BASE + 2, 12345, 70001), (2**63 + 5, 7, 33)):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        B.bitonic_keygen_i32(t, seed, start)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), W.uniform_i32(seed, n, start=start))


# -- full-size configurations ------------------------------------------------------

def _full_check(keys, asc, want_asc):
    got = gpu_sort(keys, asc)
    want = want_asc if asc else want_asc[::-1]
    assert np.array_equal(got, want)


def test_config_2_full_size():
    """n = 2^24 and n = 10,000,000 uniform, ascending (and descending)."""
    for n, seed in ((1 << 24, W.SEED_BASE + 2), (10_000_000, W.SEED_BASE + 3)):
        keys = W.uniform_i32(seed, n)
        want = O.sort_i32(keys, True)
        print(f"[case] config2 n={n}", flush=True)
        _full_check(keys, True, want)
        _full_check(keys, False, want)


@pytest.mark.parametrize("plan", [("optimized", 14, 8, 2), ("optimized", 14, 7, 2),
                                  ("optimized", 13, 6), ("optimized", 14, 10, 2),
                                  ("optimized", 15, 9, 1)],
                         ids=lambda p: "-".join(map(str, p)))
def test_wide_fusion_full_size(plan):
    """Six to ten fused steps (one-column and lane passes; the ragged size
    takes at most seven) at strides up to 2^23."""
    for n, seed in ((1 << 24, W.SEED_BASE + 2), (10_000_007, W.SEED_BASE + 3)):
        keys = W.uniform_i32(seed, n)
        want = O.sort_i32(keys, True)
        for asc in (True, False):
            print(f"[case] plan={plan} n={n} asc={asc}", flush=True)
            got = gpu_sort(keys, asc, plan)
            assert np.array_equal(got, want if asc else want[::-1]), (plan, n, asc)


@pytest.mark.parametrize("kind", W.KINDS)
def test_config_3_full_size(kind):
    """n = 2^26 per distribution, both directions, bit-exact vs the oracle."""
    n = 1 << 26
    keys = W.make_keys(kind, W.SEED_BASE + 10 + W.KINDS.index(kind), n)
    want = O.sort_i32(keys, True)
    print(f"[case] config3 kind={kind}", flush=True)
    _full_check(keys, True, want)
    _full_check(keys, False, want)


# -- segmented --------------------------------------------------------------------

def gpu_sort_segmented(keys, off, asc=True, max_seg_len=None):
    t = torch.from_numpy(np.ascontiguousarray(keys, dtype=np.int32)).cuda()
    o = torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).cuda()
    B.bitonic_sort_segmented_i32(t, o, asc, max_seg_len=max_seg_len)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_segmented_edge_lengths():
    lens = np.array([0, 1, 2, 3, 0, 5, 64, 255, 256, 257, 8191, 8192, 8193, 0, 16384,
                     16385, 65536, 65537, 100003, 1, 0], dtype=np.int64)
    off = W.offsets_from_lengths(lens) + 17   # offsets[0] != 0
    keys = W.uniform_i32(31, int(off[-1]) + 5)
    for asc in (True, False):
        got = gpu_sort_segmented(keys, off, asc)
        want = keys.copy()
        want[off[0]:off[-1]] = O.sort_segmented_i32(keys[off[0]:off[-1]], off - off[0], asc)
        assert np.array_equal(got, want), asc


def test_segmented_zero_one_principle():
    """Every 0-1 input of length n <= 16, all in one segmented call."""
    segs = []
    for n in range(1, 17):
        codes = np.arange(2**n, dtype=np.int64)
        segs.append(((codes[:, None] >> np.arange(n)) & 1).astype(np.int32).ravel())
    lens = np.concatenate([np.full(2**n, n, dtype=np.int64) for n in range(1, 17)])
    keys = np.concatenate(segs)
    off = W.offsets_from_lengths(lens)
    for asc in (True, False):
        got = gpu_sort_segmented(keys, off, asc)
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, asc)), asc


def test_segmented_config_4():
    """8192 arrays of length round(2^u), u ~ U[0, 16], uniform keys."""
    keys, off = W.batched_workload()
    for asc in (True, False):
        got = gpu_sort_segmented(keys, off, asc)
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, asc)), asc


def test_segmented_equals_looped():
    keys, off = W.batched_workload(nseg=300, seed=5, max_log2=15)
    batched = gpu_sort_segmented(keys, off, True)
    t = torch.from_numpy(keys.copy()).cuda()
    for s in range(len(off) - 1):
        B.bitonic_sort_i32(t[off[s]:off[s + 1]], True)
    torch.cuda.synchronize()
    assert np.array_equal(batched, t.cpu().numpy())


def test_segmented_big_classes_unaligned():
    """Segments spanning classes 14..21 next to tiny ones, starting at
    offsets that are not 16-byte aligned, both directions, bounded and not."""
    lens = np.array([(1 << 14) + 1, 1 << 15, (1 << 15) + 7, (1 << 17) - 3, 1 << 18, 300001,
                     (1 << 20) + 5, 5, 0, 8193, 2, (1 << 21) + 11], dtype=np.int64)
    off = W.offsets_from_lengths(lens) + 3
    keys = W.uniform_i32(41, int(off[-1]) + 9)
    for asc in (True, False):
        want = keys.copy()
        want[off[0]:off[-1]] = O.sort_segmented_i32(keys[off[0]:off[-1]], off - off[0], asc)
        assert np.array_equal(gpu_sort_segmented(keys, off, asc), want), asc
        got = gpu_sort_segmented(keys, off, asc, max_seg_len=int(lens.max()))
        assert np.array_equal(got, want), ("bounded", asc)


def test_segmented_phase_switch():
    """Phase 15 of the big segments as one launch on 2^15-key units (the
    default) and as a one-step pass and a merge: segments of 2^14 + 1 ..
    2^17 + 3 keys whose last unit is full, one key long, or past the
    segment's end (only padding), at unaligned offsets, both directions,
    uint32 and float32 keys too."""
    lens = np.array([(1 << 14) + 1, (1 << 15) - 1, 1 << 15, (1 << 15) + 1, (1 << 16) + 1,
                     (3 << 14) + 5, (1 << 17) + 3, 7, 0, (1 << 16) - 1], dtype=np.int64)
    off = W.offsets_from_lengths(lens) + 5
    keys = W.uniform_i32(43, int(off[-1]) + 3)
    saved = B.bitonic_get_tuning_value("phase_merge")
    try:
        for on in (1, 0):
            B.bitonic_set_tuning_value("phase_merge", on)
            for asc in (True, False):
                print(f"[case] segmented phase_merge={on} asc={asc}", flush=True)
                want = keys.copy()
                want[off[0]:off[-1]] = O.sort_segmented_i32(keys[off[0]:off[-1]], off - off[0], asc)
                assert np.array_equal(gpu_sort_segmented(keys, off, asc), want), (on, asc)
            bits = keys.view(np.uint32).copy()
            bits[off[3]:off[3] + len(TOTAL_ORDER_BITS)] = TOTAL_ORDER_BITS
            for kt, nk in (("uint32", O.KEY_U32), ("float32", O.KEY_F32)):
                t = torch.from_numpy(bits.view(np.int32).copy()).cuda()
                o = torch.from_numpy(off).cuda()
                B.bitonic_sort_segmented_keys(t, o, True, kt)
                torch.cuda.synchronize()
                want = bits.copy()
                view = want.view(np.float32) if kt == "float32" else want
                seg = O.sort_segmented_keys(view[off[0]:off[-1]], off - off[0], nk, True)
                want[off[0]:off[-1]] = seg.view(np.uint32)
                assert np.array_equal(t.cpu().numpy().view(np.uint32), want), (on, kt)
    finally:
        B.bitonic_set_tuning_value("phase_merge", saved)


@pytest.mark.parametrize("seg_fuse", [1, 2, 3, 4, 5])
def test_segmented_fuse_depths(seg_fuse):
    """Big-segment passes of 1..5 fused steps (4, 4, 4, 2 and 1 columns per
    thread) over classes 14..20 at an unaligned start, both directions."""
    lens = np.array([(1 << 14) + 3, (1 << 16) - 1, 1 << 17, (1 << 18) + 1, 9, (1 << 19) - 7,
                     (1 << 20) - 1, 0, 8192], dtype=np.int64)
    off = W.offsets_from_lengths(lens) + 1
    keys = W.uniform_i32(43 + seg_fuse, int(off[-1]) + 2)
    saved = B.bitonic_get_tuning_value("seg_fuse")
    try:
        B.bitonic_set_tuning_value("seg_fuse", seg_fuse)
        for asc in (True, False):
            want = keys.copy()
            want[off[0]:off[-1]] = O.sort_segmented_i32(keys[off[0]:off[-1]], off - off[0], asc)
            got = gpu_sort_segmented(keys, off, asc, max_seg_len=int(lens.max()))
            assert np.array_equal(got, want), (seg_fuse, asc)
    finally:
        B.bitonic_set_tuning_value("seg_fuse", saved)


def test_segmented_offsets_validation():
    """With validation on, a bad CSR table is refused on the device: the keys
    stay as they were and the error is recorded (1 decreasing offsets, 3 a
    segment over the bound, 4 a negative first offset); a good table sorts
    and records nothing.  The tables are checked before anything reads them
    as segments, so no kernel indexes out of range."""
    keys = W.uniform_i32(51, 4096)
    good = np.array([0, 100, 100, 3000, 4096], dtype=np.int64)
    cases = [(np.array([0, 100, 50, 4096], dtype=np.int64), None, 1),
             (good, 1000, 3),
             (np.array([-5, 100, 4000], dtype=np.int64), None, 4)]
    saved = B.bitonic_get_tuning_value("validate")
    try:
        B.bitonic_set_tuning_value("validate", 1)
        assert B.bitonic_validation_error() == 0
        for off, bound, code in cases:
            t = torch.from_numpy(keys.copy()).cuda()
            o = torch.from_numpy(off).cuda()
            print(f"[case] validation offsets={off.tolist()} bound={bound}", flush=True)
            B.bitonic_sort_segmented_i32(t, o, True, max_seg_len=bound)
            assert B.bitonic_validation_error() == code, (off, bound)
            assert np.array_equal(t.cpu().numpy(), keys)
            assert B.bitonic_validation_error() == 0     # read once, then clear
        got = gpu_sort_segmented(keys, good, True)
        assert B.bitonic_validation_error() == 0
        assert np.array_equal(got, O.sort_segmented_i32(keys, good, True))
    finally:
        B.bitonic_set_tuning_value("validate", saved)


def test_segmented_default_bound():
    """Without a bound the segmented sort bounds segments by the end of the
    keys' allocation (no device read, no wait): at least the keys it was
    given, at most 2^31, and the unbounded call sorts as the bounded one."""
    keys, off = W.batched_workload(nseg=500, seed=15, max_log2=17)
    t = torch.from_numpy(keys.copy()).cuda()
    bound = B.bitonic_segmented_default_bound(t)
    assert t.numel() <= bound <= 2**31
    if bound < 2**31:
        assert B.bitonic_segmented_default_bound(t[100:]) == bound - 100
    for asc in (True, False):
        got = gpu_sort_segmented(keys, off, asc)
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, asc)), asc


def test_segmented_pass_grid_extremes():
    """The big-segment kernels split their units into one contiguous range per
    workgroup: with 1 pass workgroup per CU a range spans many segments, with
    32 most ranges are short or empty.  Odd lengths up to 2^17."""
    keys, off = W.batched_workload(nseg=700, seed=9, max_log2=17)
    saved = B.bitonic_get_tuning_value("seg_pass_blocks_per_cu")
    try:
        want = {asc: O.sort_segmented_i32(keys, off, asc) for asc in (True, False)}
        for bpc in (1, 3, 32):
            B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", bpc)
            for asc in (True, False):
                got = gpu_sort_segmented(keys, off, asc)
                assert np.array_equal(got, want[asc]), (bpc, asc)
    finally:
        B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", saved)


def test_segmented_many_small():
    lens = (W.splitmix64(77, 0, 20000) % np.uint64(70)).astype(np.int64)
    off = W.offsets_from_lengths(lens)
    keys = W.uniform_i32(78, int(off[-1]))
    for asc in (True, False):
        got = gpu_sort_segmented(keys, off, asc, max_seg_len=int(lens.max()))
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, asc)), asc


def test_segmented_repeated_calls_reuse_scratch():
    """Calls of growing and shrinking size on one stream (scratch reuse)."""
    for nseg, seed in ((10, 1), (5000, 2), (3, 3), (9000, 4)):
        keys, off = W.batched_workload(nseg=nseg, seed=seed, max_log2=15)
        got = gpu_sort_segmented(keys, off, True)
        assert np.array_equal(got, O.sort_segmented_i32(keys, off, True)), nseg


def _hashes(t, chunk=1 << 26):
    s1 = torch.zeros((), dtype=torch.int64, device="cuda")
    s2 = torch.zeros((), dtype=torch.int64, device="cuda")
    for a in range(0, t.numel(), chunk):
        c = t[a:a + chunk].to(torch.int64)
        s1 += c.sum()
        s2 += (c * c).sum()          # wraps mod 2^64, deterministically
    return int(s1.item()), int(s2.item())


def test_wave_passes_at_2_30():
    """n = 2^30 with 2^15-key tiles, ten fused steps and lane mode 9: the
    nine- and ten-step passes of phases 25..30 spread each column over the
    four waves of a workgroup (the plan the tuning table picks beyond the
    Infinity Cache).  Checked by order, two multiset hashes, the extremes
    and sampled order statistics counted in the input."""
    n = 1 << 30
    plan = ("optimized", 15, 10)
    saved = B.bitonic_get_tuning_value("lane_pass")
    try:
        B.bitonic_set_tuning_value("lane_pass", 9)
        shapes = B.bitonic_plan_shapes(n, "keys32", plan)
        assert sum(1 for s in shapes if s["kind"] == "global_pass" and s["fuse"] == 10) >= 4
        print(f"[case] wave passes n={n} plan={plan}", flush=True)
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        B.bitonic_keygen_i32(t, W.SEED_BASE + 98)
        h0 = _hashes(t)
        lo, hi = int(t.min().item()), int(t.max().item())
        src = t.clone()
        B.bitonic_sort_plan_i32(t, True, plan)
        torch.cuda.synchronize()
        assert bool((t[1:] >= t[:-1]).all().item())
        assert _hashes(t) == h0
        assert int(t[0].item()) == lo and int(t[-1].item()) == hi
        for i in (0, n // 7, n // 2, n - 1):
            v = int(t[i].item())
            below = int((src < v).sum().item())
            upto = int((src <= v).sum().item())
            assert below <= i < upto, i
        del src, t
        torch.cuda.empty_cache()
    finally:
        B.bitonic_set_tuning_value("lane_pass", saved)


@pytest.mark.parametrize("n", [1 << 31, (1 << 31) - 1])
def test_maximum_size(n):
    """The largest supported n: sorted order, the multiset (two hashes), the
    extremes and sampled order statistics (counted independently)."""
    print(f"[case] maximum size n={n}", flush=True)
    t = torch.empty(n, dtype=torch.int32, device="cuda")
    B.bitonic_keygen_i32(t, W.SEED_BASE + 99)
    h0 = _hashes(t)
    lo, hi = int(t.min().item()), int(t.max().item())
    src = t.clone()                  # order statistics are counted in the input
    B.bitonic_sort_i32(t, True)
    torch.cuda.synchronize()
    assert bool((t[1:] >= t[:-1]).all().item())
    assert _hashes(t) == h0
    assert int(t[0].item()) == lo and int(t[-1].item()) == hi
    # the output at index i is the input's i-th order statistic:
    # #(input < v) <= i < #(input <= v)
    for i in (0, 1, n // 3, n // 2, n - 2, n - 1):
        v = int(t[i].item())
        below = int((src < v).sum().item())
        upto = int((src <= v).sum().item())
        assert below <= i < upto, i
    del src, t
    torch.cuda.empty_cache()


# -- other 32-bit key types ---------------------------------------------------------

TOTAL_ORDER_BITS = [0xFFC00001, 0xFFC00000, 0xFF800001, 0xFF800000, 0xC0000000, 0xBF800000,
                    0x80000001, 0x80000000, 0x00000000, 0x00000001, 0x3F800000, 0x40000000,
                    0x7F800000, 0x7F800001, 0x7FC00000, 0x7FC00001]


@pytest.mark.parametrize("key_type", ["uint32", "float32"])
def test_key_types(key_type):
    """Random 32-bit patterns (for float32: NaNs, infinities, subnormals and
    zeros of both signs included) and the totalOrder special values."""
    kt = O.KEY_U32 if key_type == "uint32" else O.KEY_F32
    dt = np.uint32 if key_type == "uint32" else np.float32
    special = np.array(TOTAL_ORDER_BITS * 300, dtype=np.uint32)
    for n in (3, 1000, 300001, (1 << 20) + 1):
        bits = W.uniform_i32(n + 17, n).view(np.uint32).copy()
        bits[: min(n, special.size)] = special[: min(n, special.size)]
        keys = bits.view(dt)
        for asc in (True, False):
            t = torch.from_numpy(bits.view(np.int32).copy()).cuda()
            B.bitonic_sort_keys(t, asc, key_type)
            torch.cuda.synchronize()
            want = O.sort_keys(keys, kt, asc).view(np.int32)
            assert np.array_equal(t.cpu().numpy(), want), (key_type, n, asc)


def test_key_types_segmented():
    keys, off = W.batched_workload(nseg=400, seed=12, max_log2=15)
    for key_type, kt in (("uint32", O.KEY_U32), ("float32", O.KEY_F32)):
        dt = np.uint32 if kt == O.KEY_U32 else np.float32
        for asc in (True, False):
            t = torch.from_numpy(keys.copy()).cuda()
            o = torch.from_numpy(off).cuda()
            B.bitonic_sort_segmented_keys(t, o, asc, key_type)
            torch.cuda.synchronize()
            want = O.sort_segmented_keys(keys.view(dt), off, kt, asc).view(np.int32)
            assert np.array_equal(t.cpu().numpy(), want), (key_type, asc)
