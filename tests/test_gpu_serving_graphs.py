"""GPU: the serving loop and HIP graph replays, checked against the oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_1506_01446_amd import binding as B  # noqa: E402
from paper_1506_01446_amd import serving as S  # noqa: E402
from paper_1506_01446_amd import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def _alone(r):
    t = torch.empty(r.length, dtype=torch.int32, device="cuda")
    B.bitonic_keygen_i32(t, r.key_seed)
    B.bitonic_sort_i32(t, True)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_serving_results_alone_and_in_mix():
    """The serving workload's length range (2^8 .. 2^22 keys): every request,
    packed into segmented batches, equals the oracle's sort and the same
    request sorted alone by the single-array entry point."""
    reqs = S.make_requests(0.5, 600, W.SEED_BASE + 30, min_log2=8, max_log2=22)
    assert max(r.length for r in reqs) > (1 << 21)
    ex = S.GpuExecutor(1 << 26, slots=3, max_segments=256)
    srv = S.Server(ex, 1 << 26, max_inflight=3, max_batch_segments=32, collect_results=True)
    rep = srv.run(reqs)
    print(f"[serving] {rep}", flush=True)
    assert rep["requests"] == len(reqs) and rep["failed"] == 0 and rep["rejected"] == 0
    assert rep["timed_out"] == 0 and ex.segmented_batches == rep["batches"]
    by = {r.rid: r for r in reqs}
    for c in srv.completions:
        r = by[c.rid]
        want = O.sort_i32(W.uniform_i32(r.key_seed, r.length), True)
        assert np.array_equal(c.result, want), c.rid
    for c in srv.completions[:25]:
        assert np.array_equal(_alone(by[c.rid]), c.result), c.rid


def test_graph_replays_plain_sort():
    n = (1 << 20) + 77
    buf = torch.empty(n, dtype=torch.int32, device="cuda")
    g = B.bitonic_graph_capture_sort_i32(buf, True)
    other = torch.from_numpy(W.uniform_i32(3, 50000)).cuda()
    try:
        for rep in range(4):
            keys = W.uniform_i32(100 + rep, n)
            buf.copy_(torch.from_numpy(keys))
            g.launch()
            B.bitonic_sort_i32(other, rep % 2 == 0)   # eager work between replays
            torch.cuda.synchronize()
            assert np.array_equal(buf.cpu().numpy(), O.sort_i32(keys, True)), rep
    finally:
        torch.cuda.synchronize()
        g.close()


def test_graph_replays_segmented_with_changing_table():
    cap = 64
    total = cap << 18   # room for cap segments of the maximum length
    keys_t = torch.empty(total, dtype=torch.int32, device="cuda")
    off_t = torch.zeros(cap + 1, dtype=torch.int64, device="cuda")
    g = B.bitonic_graph_capture_segmented_i32(keys_t, off_t, max_seg_len=1 << 18, ascending=False)
    try:
        for rep in range(4):
            nseg = 10 + 17 * rep
            lens = np.minimum(W.segment_lengths(rep + 5, nseg, 18.0), 1 << 18)
            off = np.zeros(cap + 1, dtype=np.int64)
            off[1:nseg + 1] = np.cumsum(lens)
            off[nseg + 1:] = off[nseg]            # unused entries: empty segments
            used = int(off[nseg])
            assert used <= total
            keys = W.uniform_i32(200 + rep, total)
            keys_t.copy_(torch.from_numpy(keys))
            off_t.copy_(torch.from_numpy(off))
            g.launch()
            torch.cuda.synchronize()
            want = keys.copy()
            want[:used] = O.sort_segmented_i32(keys[:used], off[:nseg + 1], False)
            assert np.array_equal(keys_t.cpu().numpy(), want), rep
    finally:
        torch.cuda.synchronize()
        g.close()
