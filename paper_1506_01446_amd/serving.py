"""Serving loop: continuous batching of sort requests on one GPU.

Requests arrive open-loop (Poisson); each asks to sort `length` int32 keys.
The scheduler keeps a FIFO of pending requests and at most `max_inflight`
batches on the device.  Whenever a batch slot is free and the key arena (the
HBM budget) has room, it packs pending requests, oldest first, into one
batch: a contiguous arena region holding the requests' keys back to back,
described by a CSR offset table, sorted with one segmented launch sequence
(bitonic_sort_segmented_bounded_i32) on the slot's own stream.  Batches on
different streams overlap on the device; a request that arrives while others
run is admitted as soon as a slot and memory free up (continuous batching,
not a queue drained between batches).  A request larger than the whole
budget is rejected.  Every batch, also one of a single request, goes through
the segmented sort (`pack_single=False` sends single requests to the
single-array sort instead).  A watchdog fails the requests of a batch that
has not completed `watchdog_s` seconds after its launch and retires its slot
and memory for good (the device may still be writing them), so one stuck
batch does not stall the loop.

Latency of a request = time its batch is seen complete by the host minus its
scheduled arrival time; throughput = keys sorted / wall time.

Executors: `GpuExecutor` (the HIP library; keys are generated on the device
from the request's seed, stay there until completion, and can be copied back
for checking) and `FakeExecutor` (CPU, for tests of the scheduler: sorts with
numpy and completes after a simulated duration).
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import gc
import time

import numpy as np

from . import workloads as W


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds from the start of the run
    length: int
    key_seed: int


@dataclasses.dataclass
class Completion:
    rid: int
    arrival: float
    admitted: float
    done: float
    length: int
    batch: int
    result: np.ndarray | None = None


class Arena:
    """First-fit allocator over [0, capacity) keys; regions start at
    multiples of `align` keys."""

    def __init__(self, capacity: int, align: int = 64):
        self.capacity = int(capacity)
        self.align = align
        self.free_list = [(0, self.capacity)]   # sorted (start, size)
        self.used = 0
        self.peak = 0

    def alloc(self, n: int):
        n = max(self.align, -(-int(n) // self.align) * self.align)
        for i, (s, sz) in enumerate(self.free_list):
            if sz >= n:
                if sz == n:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (s + n, sz - n)
                self.used += n
                self.peak = max(self.peak, self.used)
                return s, n
        return None

    def free(self, start: int, n: int) -> None:
        self.used -= n
        i = bisect.bisect_left(self.free_list, (start, 0))
        self.free_list.insert(i, (start, n))
        # coalesce neighbours
        merged = []
        for s, sz in self.free_list:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + sz)
            else:
                merged.append((s, sz))
        self.free_list = merged


@dataclasses.dataclass
class Batch:
    bid: int
    requests: list
    offsets: np.ndarray       # CSR offsets relative to the region start
    region: tuple             # (start, size) in the arena
    admitted: float
    handle: object = None
    launched: float = 0.0


class FakeExecutor:
    """CPU stand-in for tests: sorts with numpy and reports completion after
    `latency_s + keys / rate` of (virtual) time."""

    def __init__(self, rate_keys_per_s: float = 1e9, latency_s: float = 1e-4,
                 fail_batches: set | None = None, clock=None, hang_batches: set | None = None):
        self.rate = rate_keys_per_s
        self.latency = latency_s
        self.fail = set(fail_batches or ())
        self.hang = set(hang_batches or ())   # batches that never complete
        self.abandoned = []
        self.clock = clock
        self.inflight_peak = 0
        self._inflight = 0
        self.arena_keys = {}

    def submit(self, batch: Batch, now: float, ascending: bool):
        if batch.bid in self.fail:
            raise RuntimeError(f"batch {batch.bid} failed to launch")
        self._inflight += 1
        self.inflight_peak = max(self.inflight_peak, self._inflight)
        total = int(batch.offsets[-1])
        outs = []
        for r, a, b in zip(batch.requests, batch.offsets[:-1], batch.offsets[1:]):
            k = np.sort(W.uniform_i32(r.key_seed, r.length))
            outs.append(k if ascending else k[::-1].copy())
        ready = float("inf") if batch.bid in self.hang else now + self.latency + total / self.rate
        return {"ready": ready, "outs": outs, "bid": batch.bid}

    def poll(self, handle, now: float) -> bool:
        done = now >= handle["ready"]
        if done:
            self._inflight -= 1
        return done

    def abandon(self, handle) -> None:
        self._inflight -= 1
        self.abandoned.append(handle["bid"])

    def result(self, handle, i: int) -> np.ndarray:
        return handle["outs"][i]


class GpuExecutor:
    """The HIP library on one GPU: one stream per in-flight slot, keys
    generated on the device into the arena, one segmented sort per batch."""

    def __init__(self, capacity_keys: int, slots: int, max_segments: int, keep_results=False,
                 pack_single: bool = True):
        import torch

        from . import binding as B
        self.torch = torch
        self.B = B
        B.load()
        self.arena = torch.empty(int(capacity_keys), dtype=torch.int32, device="cuda")
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.free_slots = list(range(slots))
        self.off_dev = [torch.empty(max_segments + 1, dtype=torch.int64, device="cuda")
                        for _ in range(slots)]
        self.off_host = [torch.empty(max_segments + 1, dtype=torch.int64, pin_memory=True)
                         for _ in range(slots)]
        self.keep = keep_results
        self.pack_single = pack_single
        self.segmented_batches = 0
        self.lib = B.load()

    def submit(self, batch: Batch, now: float, ascending: bool):
        torch, B = self.torch, self.B
        slot = self.free_slots.pop()
        st = self.streams[slot]
        start, _ = batch.region
        nseg = len(batch.requests)
        oh = self.off_host[slot]
        oh[:nseg + 1] = torch.from_numpy(batch.offsets)
        od = self.off_dev[slot]
        base = self.arena.data_ptr() + 4 * start
        sp = st.cuda_stream
        with torch.cuda.stream(st):
            od[:nseg + 1].copy_(oh[:nseg + 1], non_blocking=True)
        for r, a in zip(batch.requests, batch.offsets[:-1]):
            rc = self.lib.bitonic_keygen_i32(base + 4 * int(a), r.length, r.key_seed & (2**64 - 1),
                                             0, sp)
            if rc:
                raise B.BitonicError("bitonic_keygen_i32", rc)
        max_len = max(r.length for r in batch.requests)
        if nseg == 1 and max_len > 1 and not self.pack_single:
            rc = self.lib.bitonic_sort_i32(base, max_len, int(ascending), sp)
            name = "bitonic_sort_i32"
        else:
            rc = self.lib.bitonic_sort_segmented_bounded_i32(base, od.data_ptr(), nseg,
                                                             max(max_len, 1), int(ascending), sp)
            name = "bitonic_sort_segmented_bounded_i32"
            self.segmented_batches += 1
        if rc:
            raise B.BitonicError(name, rc)
        ev = torch.cuda.Event()
        ev.record(st)
        return {"slot": slot, "event": ev, "start": start, "offsets": batch.offsets}

    def poll(self, handle, now: float) -> bool:
        if handle["event"].query():
            self.free_slots.append(handle["slot"])
            return True
        return False

    def abandon(self, handle) -> None:
        """A batch the watchdog gave up on: its stream (and slot) is not
        reused, since work queued behind it would wait for it."""
        self.abandoned = getattr(self, "abandoned", []) + [handle["slot"]]

    def result(self, handle, i: int) -> np.ndarray:
        a = handle["start"] + int(handle["offsets"][i])
        b = handle["start"] + int(handle["offsets"][i + 1])
        return self.arena[a:b].cpu().numpy()


class Server:
    def __init__(self, executor, budget_keys: int, max_inflight: int = 3,
                 max_batch_keys: int = 1 << 26, max_batch_segments: int = 1024,
                 ascending: bool = True, collect_results: bool = False,
                 watchdog_s: float = 10.0):
        self.ex = executor
        self.arena = Arena(budget_keys)
        self.max_inflight = max_inflight
        self.watchdog_s = watchdog_s
        self.timed_out: list[Request] = []
        self.queue_samples = 0
        self.queue_sum = 0
        self.queue_peak = 0
        self.max_batch_keys = max_batch_keys
        self.max_batch_segments = max_batch_segments
        self.ascending = ascending
        self.collect = collect_results
        self.pending = collections.deque()
        self.inflight: list[Batch] = []
        self.completions: list[Completion] = []
        self.rejected: list[Request] = []
        self.failed: list[Request] = []
        self.batches = 0
        self.inflight_peak = 0

    def _form_batch(self, now: float):
        reqs, total = [], 0
        while self.pending and len(reqs) < self.max_batch_segments:
            r = self.pending[0]
            if reqs and total + r.length > self.max_batch_keys:
                break
            reqs.append(r)
            total += r.length
            self.pending.popleft()
        if not reqs:
            return None
        region = self.arena.alloc(total)
        while region is None and len(reqs) > 1:   # shrink until it fits
            self.pending.appendleft(reqs.pop())
            total = sum(r.length for r in reqs)
            region = self.arena.alloc(total)
        if region is None:                        # wait for memory
            for r in reversed(reqs):
                self.pending.appendleft(r)
            return None
        off = np.zeros(len(reqs) + 1, dtype=np.int64)
        np.cumsum([r.length for r in reqs], out=off[1:])
        b = Batch(self.batches, reqs, off, region, now)
        self.batches += 1
        return b

    def _admit(self, now: float) -> None:
        while self.pending and len(self.inflight) < self.max_inflight:
            b = self._form_batch(now)
            if b is None:
                return
            try:
                b.handle = self.ex.submit(b, now, self.ascending)
            except Exception:
                self.arena.free(*b.region)
                self.failed.extend(b.requests)
                continue
            b.launched = now
            self.inflight.append(b)
            self.inflight_peak = max(self.inflight_peak, len(self.inflight))

    def _reap(self, now: float) -> None:
        still = []
        for b in self.inflight:
            if self.ex.poll(b.handle, now):
                for i, r in enumerate(b.requests):
                    res = self.ex.result(b.handle, i) if self.collect else None
                    self.completions.append(Completion(r.rid, r.arrival, b.admitted, now,
                                                       r.length, b.bid, res))
                self.arena.free(*b.region)
            elif now - b.launched > self.watchdog_s:
                # never completed: fail its requests; its memory and slot stay
                # retired (the device may still write them)
                self.ex.abandon(b.handle)
                self.timed_out.extend(b.requests)
                self.max_inflight -= 1
            else:
                still.append(b)
        self.inflight = still

    def run(self, requests: list, clock=None, idle_sleep: float = 2e-5, sleep=None) -> dict:
        """Serve `requests` (sorted by arrival).  `clock()` returns seconds
        since the start (default: wall clock); `sleep(dt)` waits."""
        t0 = time.perf_counter()
        clock = clock or (lambda: time.perf_counter() - t0)
        sleep = sleep or time.sleep
        i = 0
        n = len(requests)
        while i < n or self.pending or self.inflight:
            now = clock()
            while i < n and requests[i].arrival <= now:
                r = requests[i]
                if r.length > self.arena.capacity:
                    self.rejected.append(r)
                else:
                    self.pending.append(r)
                i += 1
            self._reap(now)
            self._admit(now)
            if self.max_inflight <= 0:        # every slot retired by the watchdog
                self.timed_out.extend(self.pending)
                self.pending.clear()
                self.timed_out.extend(requests[i:])
                i = n
            q = len(self.pending)
            self.queue_samples += 1
            self.queue_sum += q
            self.queue_peak = max(self.queue_peak, q)
            if i < n and not self.pending and not self.inflight:
                wait = requests[i].arrival - clock()
                if wait > 0:
                    sleep(min(wait, 1e-3))
            else:
                sleep(idle_sleep)
        wall = clock()
        return self.report(wall)

    def report(self, wall: float) -> dict:
        lat = np.array([c.done - c.arrival for c in self.completions]) * 1e3
        keys = sum(c.length for c in self.completions)
        pct = (lambda q: float(np.percentile(lat, q))) if len(lat) else (lambda q: None)
        return {"requests": len(self.completions), "rejected": len(self.rejected),
                "failed": len(self.failed), "timed_out": len(self.timed_out),
                "batches": self.batches,
                "queue_depth_peak": self.queue_peak,
                "queue_depth_mean": round(self.queue_sum / max(1, self.queue_samples), 3),
                "mean_batch": round(len(self.completions) / max(1, self.batches), 2),
                "inflight_peak": self.inflight_peak,
                "arena_peak_keys": self.arena.peak,
                "wall_s": round(wall, 3),
                "p50_ms": None if not len(lat) else round(pct(50), 3),
                "p99_ms": None if not len(lat) else round(pct(99), 3),
                "p999_ms": None if not len(lat) else round(pct(99.9), 3),
                "mean_ms": None if not len(lat) else round(float(lat.mean()), 3),
                "gkeys_s": round(keys / max(wall, 1e-9) / 1e9, 4)}


def make_requests(duration_s: float, rate: float, seed: int, min_log2=8.0, max_log2=22.0):
    t, lens, seeds = W.serving_requests(duration_s, rate, seed, min_log2, max_log2)
    return [Request(i, float(a), int(n), int(s)) for i, (a, n, s) in enumerate(zip(t, lens, seeds))]


def run_gpu(duration_s: float = 60.0, rate: float = 2000.0, budget_bytes: int = 32 << 30,
            slots: int = 3, seed: int = W.SEED_BASE + 30, pack_single: bool = True) -> dict:
    """The serving workload: Poisson arrivals at `rate`, lengths log-uniform
    in [2^8, 2^22], keys uniform; `budget_bytes` of HBM for keys."""
    reqs = make_requests(duration_s, rate, seed)
    budget = budget_bytes // 4
    ex = GpuExecutor(budget, slots, max_segments=1024, pack_single=pack_single)
    # warm the kernels and the per-stream scratch once before the clock starts
    warm = Server(ex, budget, max_inflight=slots)
    warm.run([Request(-1 - k, 0.0, 1 << 20, 7 + k) for k in range(slots * 2)])
    srv = Server(ex, budget, max_inflight=slots)
    ex.segmented_batches = 0
    # The request list (all arrivals of the run) is built up front; move it
    # out of the collector's reach, so that a full collection during the run
    # does not walk it and stall the loop for milliseconds.
    gc.collect()
    gc.freeze()
    try:
        out = srv.run(reqs)
    finally:
        gc.unfreeze()
    out.update({"segmented_batches": ex.segmented_batches,
                "duration_s": duration_s, "rate_per_s": rate, "budget_bytes": budget_bytes,
                "streams": slots, "offered_gkeys_s":
                round(sum(r.length for r in reqs) / duration_s / 1e9, 4)})
    return out
