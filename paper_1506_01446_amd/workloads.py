"""Seeded synthetic inputs for the bitonic sort workloads.

This module only draws numbers.  It holds no step of the sorting method, so
both the CPU oracle tests and the HIP path may take their inputs from it.

Every stream is counter based: value ``i`` of stream ``seed`` is
``splitmix64(seed + (i + 1) * GAMMA)``, the SplitMix64 generator of Steele,
Lea and Flood ("Fast splittable pseudorandom number generators", OOPSLA
2014), so any slice of a stream can be produced without the rest, on the host
here or on the device by the library's ``keygen`` kernel.

Workloads (the paper measures 32-bit random integers, powers of two from
128K to 256M keys, section 5):

* ``uniform``   key_i = high 32 bits of the stream word, read as signed int32
* ``sorted``    the uniform array in ascending order
* ``reverse``   the uniform array in descending order
* ``distinct16`` 16 distinct int32 values drawn uniformly (repeats rejected),
  every key picks one of them uniformly
* ``equal``     every key is one seeded int32 value
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Seed base for the workloads; each configuration adds its own offset.
SEED_BASE = 1506014460

KINDS = ("uniform", "sorted", "reverse", "distinct16", "equal")


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Words ``start .. start+count-1`` of the counter-based stream ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_scalar(seed: int, i: int) -> int:
    """Word ``i`` of stream ``seed``, in plain Python integers (for tests)."""
    mask = (1 << 64) - 1
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & mask
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
    return z ^ (z >> 31)


def uniform_i32(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Keys uniform over the full signed int32 range."""
    w = splitmix64(seed, start, n)
    return (w >> np.uint64(32)).astype(np.uint32).view(np.int32)


def uniform_i64(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Keys uniform over the full signed int64 range (the whole 64-bit word)."""
    return splitmix64(seed, start, n).view(np.int64)


def unit_doubles(seed: int, n: int, start: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits of each word."""
    w = splitmix64(seed, start, n)
    return (w >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))


def make_keys(kind: str, seed: int, n: int) -> np.ndarray:
    """One input array of ``n`` int32 keys of the given distribution."""
    if kind == "uniform":
        return uniform_i32(seed, n)
    if kind == "sorted":
        return np.sort(uniform_i32(seed, n), kind="stable")
    if kind == "reverse":
        return np.sort(uniform_i32(seed, n), kind="stable")[::-1].copy()
    if kind == "distinct16":
        values: list[int] = []
        j = 0
        while len(values) < 16:
            v = int(uniform_i32(seed, 1, start=j)[0])
            j += 1
            if v not in values:
                values.append(v)
        pick = (splitmix64(seed ^ 0x5A5A5A5A, 0, n) >> np.uint64(60)).astype(np.int64)
        return np.asarray(values, dtype=np.int32)[pick]
    if kind == "equal":
        return np.full(n, uniform_i32(seed, 1)[0], dtype=np.int32)
    raise ValueError(f"unknown key distribution {kind!r}")


def segment_lengths(seed: int, nseg: int, max_log2: float = 16.0) -> np.ndarray:
    """Lengths ``round(2**u)`` with ``u`` uniform in ``[0, max_log2]``."""
    u = unit_doubles(seed, nseg) * max_log2
    return np.floor(np.exp2(u) + 0.5).astype(np.int64)


def offsets_from_lengths(lengths: np.ndarray) -> np.ndarray:
    """CSR offsets (``nseg + 1`` entries, int64) for contiguous segments."""
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def batched_workload(nseg: int = 8192, seed: int = SEED_BASE + 20,
                     max_log2: float = 16.0):
    """Segment table plus keys for the batched segmented sort workload:
    ``nseg`` arrays whose lengths are 2**u rounded, u uniform in
    [0, max_log2], keys uniform over the int32 range."""
    lens = segment_lengths(seed, nseg, max_log2)
    off = offsets_from_lengths(lens)
    keys = uniform_i32(seed + 1, int(off[-1]))
    return keys, off


def serving_requests(duration_s: float, rate_per_s: float, seed: int,
                     min_log2: float = 8.0, max_log2: float = 22.0):
    """Open-loop Poisson arrivals: (arrival time in s, length, key seed).

    Gaps are exponential with mean ``1/rate``; lengths are log-uniform in
    ``[2**min_log2, 2**max_log2]`` rounded to an integer.  Request ``r``
    carries keys ``uniform_i32(key_seed_r, length)``.
    """
    expected = int(duration_s * rate_per_s * 1.5) + 64
    gaps = -np.log1p(-unit_doubles(seed, expected)) / rate_per_s
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    m = len(t)
    u = unit_doubles(seed + 1, m)
    lens = np.floor(np.exp2(min_log2 + (max_log2 - min_log2) * u) + 0.5).astype(np.int64)
    key_seeds = (np.int64(seed + 2) * 1_000_003 + np.arange(m, dtype=np.int64))
    return t, lens, key_seeds


__all__ = [
    "GAMMA", "SEED_BASE", "KINDS", "splitmix64", "splitmix64_scalar", "uniform_i64",
    "uniform_i32", "unit_doubles", "make_keys", "segment_lengths",
    "offsets_from_lengths", "batched_workload", "serving_requests",
]
