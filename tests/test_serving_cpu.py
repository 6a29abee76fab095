"""Serving scheduler on the CPU with a fake executor and a virtual clock:
admission under the memory budget, overlap of batches, continuous batching,
rejection of oversize requests, failure isolation, and results equal to a
plain sort whether a request is served alone or in a mix."""
import numpy as np
import pytest

from paper_1506_01446_amd import serving as S
from paper_1506_01446_amd import workloads as W


class VClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


def _serve(reqs, budget=1 << 24, inflight=3, rate=1e9, latency=1e-4, fail=None, **kw):
    clk = VClock()
    ex = S.FakeExecutor(rate, latency, fail_batches=fail)
    srv = S.Server(ex, budget, max_inflight=inflight, collect_results=True, **kw)
    rep = srv.run(reqs, clock=clk.now, sleep=clk.sleep)
    return srv, ex, rep


def test_arena_alloc_free_coalesce():
    a = S.Arena(1024, align=64)
    r1 = a.alloc(10)
    r2 = a.alloc(100)
    r3 = a.alloc(64)
    assert r1 == (0, 64) and r2 == (64, 128) and r3 == (192, 64)
    assert a.alloc(1024) is None
    a.free(*r2)
    assert a.alloc(128) == (64, 128)
    a.free(*r1)
    a.free(64, 128)
    a.free(*r3)
    assert a.free_list == [(0, 1024)] and a.used == 0
    assert a.peak == 256


def test_all_requests_sorted():
    reqs = S.make_requests(0.05, 2000, 3, min_log2=4, max_log2=12)
    srv, _, rep = _serve(reqs)
    assert rep["requests"] == len(reqs) and rep["rejected"] == 0
    by = {r.rid: r for r in reqs}
    for c in srv.completions:
        r = by[c.rid]
        assert np.array_equal(c.result, np.sort(W.uniform_i32(r.key_seed, r.length)))
        assert c.done >= c.admitted >= c.arrival - 1e-12


def test_budget_and_oversize_rejection():
    reqs = [S.Request(0, 0.0, 5000, 1), S.Request(1, 0.0, 3000, 2),
            S.Request(2, 0.0, 9000, 3), S.Request(3, 0.001, 100, 4)]
    srv, _, rep = _serve(reqs, budget=8192, rate=1e6, inflight=2, max_batch_keys=5000)
    assert [r.rid for r in srv.rejected] == [2]
    assert srv.arena.peak <= 8192
    assert sorted(c.rid for c in srv.completions) == [0, 1, 3]


def test_batches_overlap_and_continuous_admission():
    # slow device: several batches in flight; a late arrival is admitted while
    # earlier batches still run
    reqs = [S.Request(i, 0.0001 * i, 1 << 14, i + 10) for i in range(8)]
    srv, ex, rep = _serve(reqs, rate=1e8, latency=2e-3, inflight=3, max_batch_segments=1)
    assert rep["inflight_peak"] == 3 and ex.inflight_peak == 3
    comp = {c.rid: c for c in srv.completions}
    first_done = min(c.done for c in comp.values())
    assert any(c.admitted < first_done and c.arrival > 0 for c in comp.values())
    # a request admitted after another was completed reuses its slot
    assert any(c.admitted >= first_done for c in comp.values())


def test_failure_isolated():
    reqs = [S.Request(i, 0.001 * i, 1000, i) for i in range(6)]
    srv, _, rep = _serve(reqs, fail={2}, max_batch_segments=1, inflight=1)
    assert len(srv.failed) == 1 and srv.failed[0].rid == 2
    assert sorted(c.rid for c in srv.completions) == [0, 1, 3, 4, 5]


def test_same_result_alone_and_in_mix():
    reqs = S.make_requests(0.02, 5000, 9, min_log2=5, max_log2=11)
    srv_mix, _, _ = _serve(reqs, max_batch_segments=64, latency=1e-3)
    mix = {c.rid: c.result for c in srv_mix.completions}
    assert max(c.batch for c in srv_mix.completions) < len(reqs) - 1  # batches really mixed
    for r in reqs[:20]:
        srv_one, _, _ = _serve([S.Request(r.rid, 0.0, r.length, r.key_seed)])
        assert np.array_equal(srv_one.completions[0].result, mix[r.rid])


def test_report_fields():
    reqs = S.make_requests(0.02, 1000, 4, min_log2=4, max_log2=8)
    _, _, rep = _serve(reqs)
    for k in ("p50_ms", "p99_ms", "gkeys_s", "batches", "inflight_peak"):
        assert k in rep
    assert rep["p99_ms"] >= rep["p50_ms"] >= 0


def test_watchdog_fails_stuck_batch_and_continues():
    """A batch that never completes: the watchdog fails its requests after
    watchdog_s, retires its slot and memory, and the loop serves the rest."""
    reqs = [S.Request(i, 0.001 * i, 1000, i) for i in range(8)]
    clk = VClock()
    ex = S.FakeExecutor(1e9, 1e-4, hang_batches={2})
    srv = S.Server(ex, 1 << 20, max_inflight=2, max_batch_segments=1, collect_results=True,
                   watchdog_s=0.05)
    rep = srv.run(reqs, clock=clk.now, sleep=clk.sleep)
    assert [r.rid for r in srv.timed_out] == [2] and rep["timed_out"] == 1
    assert ex.abandoned == [2]
    assert sorted(c.rid for c in srv.completions) == [0, 1, 3, 4, 5, 6, 7]
    assert srv.arena.used == 1024        # the stuck batch's region stays retired
    for c in srv.completions:
        assert np.array_equal(c.result, np.sort(W.uniform_i32(c.rid, 1000)))


def test_watchdog_every_slot_stuck_ends_the_run():
    """If every slot is retired the loop ends, failing what is left."""
    reqs = [S.Request(i, 0.0, 100, i) for i in range(5)]
    clk = VClock()
    ex = S.FakeExecutor(1e9, 1e-4, hang_batches={0, 1})
    srv = S.Server(ex, 1 << 20, max_inflight=2, max_batch_segments=1, watchdog_s=0.01)
    rep = srv.run(reqs, clock=clk.now, sleep=clk.sleep)
    assert rep["requests"] == 0 and rep["timed_out"] == 5


def test_queue_depth_reported():
    reqs = [S.Request(i, 0.0, 1 << 14, i) for i in range(20)]
    _, _, rep = _serve(reqs, rate=1e8, latency=1e-3, inflight=1, max_batch_segments=2)
    assert rep["queue_depth_peak"] >= 10 and rep["queue_depth_mean"] > 0
