"""Python face of the CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import this module.  It loads ``liboracle.so`` (built by
``oracle/build_oracle.py`` with g++) and never touches the HIP library.

* :func:`sort_i32`, :func:`sort_segmented_i32` -- the plain definition: keys
  in signed int32 order, descending read backwards (section 3 of the paper
  defines the sort; std::sort stands in for the CPU QuickSort of section 5).
* :func:`bitonic_i32` -- the scalar bitonic network of sections 3.1-3.3, in
  the paper's phase/step order, with step and compare-exchange counters and a
  per-step hook.  ``variant`` is one of :data:`STANDARD`, :data:`FLIP`,
  :data:`FLIP_VIRTUAL` (see the C source for their definitions).
* :func:`sort_keys`, :func:`sort_keys64`, :func:`sort_pairs` -- the plain
  definitions for the other key types and for (key, value) pairs.
* :func:`bitonic_merge_i32` -- the bitonic merge of section 3.1 alone.
* :func:`step_pairs` -- the comparators of one step.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

STANDARD, FLIP, FLIP_VIRTUAL = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

_HOOK = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_int32), ctypes.c_int64)

_lib = None


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    p32 = ctypes.POINTER(ctypes.c_int32)
    p64 = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_sort_i32.argtypes = [p32, ctypes.c_int64, ctypes.c_int]
    lib.oracle_sort_i32.restype = ctypes.c_int
    lib.oracle_sort_i32_parallel.argtypes = [p32, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
    lib.oracle_sort_i32_parallel.restype = ctypes.c_int
    lib.oracle_sort_segmented_i32.argtypes = [p32, p64, ctypes.c_int64, ctypes.c_int]
    lib.oracle_sort_segmented_i32.restype = ctypes.c_int
    lib.oracle_bitonic_i32.argtypes = [p32, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                       _HOOK, ctypes.c_void_p, p64, p64]
    lib.oracle_bitonic_i32.restype = ctypes.c_int
    lib.oracle_step_pairs.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_int, p64, p64,
                                      ctypes.POINTER(ctypes.c_int8), ctypes.c_int64]
    lib.oracle_step_pairs.restype = ctypes.c_int64
    lib.oracle_bitonic_merge_i32.argtypes = [p32, ctypes.c_int64]
    lib.oracle_bitonic_merge_i32.restype = ctypes.c_int
    lib.oracle_bitonic_segmented_i32.argtypes = [p32, p64, ctypes.c_int64, ctypes.c_int]
    lib.oracle_bitonic_segmented_i32.restype = ctypes.c_int
    lib.oracle_bitonic_batch_i32.argtypes = [p32, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_int, ctypes.c_int]
    lib.oracle_bitonic_batch_i32.restype = ctypes.c_int
    pu = ctypes.POINTER(ctypes.c_uint32)
    lib.oracle_sort_u32.argtypes = [pu, ctypes.c_int64, ctypes.c_int]
    lib.oracle_sort_u32.restype = ctypes.c_int
    lib.oracle_sort_f32_bits.argtypes = [pu, ctypes.c_int64, ctypes.c_int]
    lib.oracle_sort_f32_bits.restype = ctypes.c_int
    lib.oracle_sort_segmented_keys.argtypes = [pu, p64, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
    lib.oracle_sort_segmented_keys.restype = ctypes.c_int
    lib.oracle_sort_keys64.argtypes = [ctypes.POINTER(ctypes.c_uint64), ctypes.c_int64,
                                       ctypes.c_int, ctypes.c_int]
    lib.oracle_sort_keys64.restype = ctypes.c_int
    lib.oracle_sort_pairs.argtypes = [pu, p32, ctypes.c_int64, ctypes.c_int, ctypes.c_int]
    lib.oracle_sort_pairs.restype = ctypes.c_int
    lib.oracle_mutant_id.argtypes = []
    lib.oracle_mutant_id.restype = ctypes.c_int
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """The oracle library (built on first use if absent)."""
    global _lib
    if path is not None:
        return _bind(ctypes.CDLL(path))
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build_oracle
            build_oracle.build()
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _keys(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32)).copy()


def sort_i32(keys, ascending: bool = True, lib=None) -> np.ndarray:
    """The plain definition: a sorted copy of ``keys``."""
    lib = lib or load()
    x = _keys(keys)
    rc = lib.oracle_sort_i32(_p32(x), x.size, int(bool(ascending)))
    if rc:
        raise ValueError("oracle_sort_i32 rejected its arguments")
    return x


KEY_I32, KEY_U32, KEY_F32 = 0, 1, 2
_KEY_DTYPES = {KEY_I32: np.int32, KEY_U32: np.uint32, KEY_F32: np.float32}


def sort_i32_parallel(keys, ascending: bool = True, threads: int = 1, lib=None) -> np.ndarray:
    """sort_i32 on `threads` host threads (chunks sorted in parallel, then
    merged pairwise): a CPU baseline on all cores."""
    lib = lib or load()
    x = _keys(keys)
    if lib.oracle_sort_i32_parallel(_p32(x), x.size, int(bool(ascending)), int(threads)):
        raise ValueError("oracle_sort_i32_parallel rejected its arguments")
    return x


def sort_keys(keys, key_type: int, ascending: bool = True, lib=None) -> np.ndarray:
    """Plain definition for int32 / uint32 / float32 keys (float32 in IEEE
    totalOrder).  Returns an array of the key type (bit-exact)."""
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(keys, dtype=_KEY_DTYPES[key_type])).copy()
    bits = x.view(np.uint32)
    fn = {KEY_I32: None, KEY_U32: lib.oracle_sort_u32, KEY_F32: lib.oracle_sort_f32_bits}[key_type]
    if fn is None:
        return sort_i32(x, ascending, lib).view(np.int32)
    if fn(bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), x.size, int(bool(ascending))):
        raise ValueError("oracle rejected its arguments")
    return x


KEY_I64, KEY_U64, KEY_F64 = 3, 4, 5
_KEY64_DTYPES = {KEY_I64: np.int64, KEY_U64: np.uint64, KEY_F64: np.float64}


def sort_keys64(keys, key_type: int, ascending: bool = True, lib=None) -> np.ndarray:
    """Plain definition for int64 / uint64 / float64 keys (float64 in IEEE
    totalOrder).  Returns an array of the key type (bit-exact)."""
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(keys, dtype=_KEY64_DTYPES[key_type])).copy()
    bits = x.view(np.uint64)
    if lib.oracle_sort_keys64(bits.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), x.size,
                              int(key_type), int(bool(ascending))):
        raise ValueError("oracle rejected its arguments")
    return x


def sort_pairs(keys, values, key_type: int = KEY_I32, ascending: bool = True, lib=None):
    """Plain definition of the key-value sort: by key (key_type 0..2, in the
    requested direction), equal keys by int32 value ascending.  Returns
    (keys, values) as new arrays."""
    lib = lib or load()
    k = np.ascontiguousarray(np.asarray(keys, dtype=_KEY_DTYPES[key_type])).copy()
    v = np.ascontiguousarray(np.asarray(values, dtype=np.int32)).copy()
    if k.size != v.size:
        raise ValueError("keys and values differ in length")
    if lib.oracle_sort_pairs(k.view(np.uint32).ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                             _p32(v), k.size, int(key_type), int(bool(ascending))):
        raise ValueError("oracle rejected its arguments")
    return k, v


def sort_segmented_keys(keys, offsets, key_type: int, ascending: bool = True, lib=None):
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(keys, dtype=_KEY_DTYPES[key_type])).copy()
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if lib.oracle_sort_segmented_keys(x.view(np.uint32).ctypes.data_as(
            ctypes.POINTER(ctypes.c_uint32)), _p64(off), off.size - 1, int(key_type),
            int(bool(ascending))):
        raise ValueError("oracle rejected its arguments")
    return x


def sort_segmented_i32(keys, offsets, ascending: bool = True, lib=None) -> np.ndarray:
    """Plain definition applied to every segment of a CSR table."""
    lib = lib or load()
    x = _keys(keys)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.size < 1 or off[-1] > x.size or off[0] < 0:
        raise ValueError("offsets out of range")
    rc = lib.oracle_sort_segmented_i32(_p32(x), _p64(off), off.size - 1,
                                       int(bool(ascending)))
    if rc:
        raise ValueError("oracle_sort_segmented_i32 rejected its arguments")
    return x


def bitonic_i32(keys, ascending: bool = True, variant: int = FLIP_VIRTUAL,
                hook=None, lib=None):
    """Scalar network.  Returns ``(sorted copy, steps, compare-exchanges)``.

    ``hook(phase, step, state)`` is called after every step with a copy of
    the working array (padded to N for the materialised variants).
    """
    lib = lib or load()
    x = _keys(keys)
    steps = np.zeros(1, dtype=np.int64)
    cmps = np.zeros(1, dtype=np.int64)
    if hook is None:
        cb = ctypes.cast(None, _HOOK)
    else:
        def _cb(_ctx, phase, step, ptr, length):
            hook(phase, step, np.ctypeslib.as_array(ptr, shape=(length,)).copy()
                 if length > 0 else np.zeros(0, np.int32))
        cb = _HOOK(_cb)
    rc = lib.oracle_bitonic_i32(_p32(x), x.size, int(bool(ascending)), int(variant),
                                cb, None, _p64(steps), _p64(cmps))
    if rc:
        raise ValueError("oracle_bitonic_i32 rejected its arguments")
    return x, int(steps[0]), int(cmps[0])


def bitonic_segmented_i32(keys, offsets, ascending: bool = True, lib=None) -> np.ndarray:
    lib = lib or load()
    x = _keys(keys)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    rc = lib.oracle_bitonic_segmented_i32(_p32(x), _p64(off), off.size - 1,
                                          int(bool(ascending)))
    if rc:
        raise ValueError("oracle_bitonic_segmented_i32 rejected its arguments")
    return x


def bitonic_batch_i32(arrays: np.ndarray, ascending: bool = True,
                      variant: int = FLIP_VIRTUAL, lib=None) -> np.ndarray:
    """Scalar network on every row of a 2-D ``(count, n)`` array."""
    lib = lib or load()
    x = np.ascontiguousarray(np.asarray(arrays, dtype=np.int32)).copy()
    count, n = x.shape
    if lib.oracle_bitonic_batch_i32(_p32(x), n, count, int(bool(ascending)), int(variant)):
        raise ValueError("oracle_bitonic_batch_i32 rejected its arguments")
    return x


def bitonic_merge_i32(seq, lib=None) -> np.ndarray:
    """Bitonic merge (half-cleaner cascade) of one power-of-two sequence."""
    lib = lib or load()
    x = _keys(seq)
    if lib.oracle_bitonic_merge_i32(_p32(x), x.size):
        raise ValueError("length must be a power of two")
    return x


def step_pairs(N: int, variant: int, phase: int, step: int, lib=None):
    """Comparators ``[(lo, hi, smaller_to_lo)]`` of one network step."""
    lib = lib or load()
    m = lib.oracle_step_pairs(N, variant, phase, step, None, None, None, 0)
    if m < 0:
        raise ValueError("bad step")
    lo = np.zeros(m, np.int64)
    hi = np.zeros(m, np.int64)
    up = np.zeros(m, np.int8)
    lib.oracle_step_pairs(N, variant, phase, step, _p64(lo), _p64(hi),
                          up.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), m)
    return [(int(a), int(b), bool(c)) for a, b, c in zip(lo, hi, up)]
