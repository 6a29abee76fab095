"""Thin Python binding of libbitonic_mi355x.so (include/bitonic.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, checks that tensors are contiguous int32 / int64 device
tensors, passes their device pointers and the current HIP stream, and turns
a nonzero status into :class:`BitonicError`.  All sorting work runs in the
library's HIP kernels; there is no fallback.  If the library has not been
built, loading it raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbitonic_mi355x.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bitonic.h")

PLAN_KINDS = {"auto": 0, "basic": 1, "semi": 2, "optimized": 3}
STATUS = {0: "BITONIC_OK", -1: "BITONIC_EINVAL", -2: "BITONIC_ENOMEM",
          -3: "BITONIC_ELAUNCH", -4: "BITONIC_EUNSUPPORTED", -5: "BITONIC_EDEVICE"}


class BitonicError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        super().__init__(f"{fn} failed: {status} ({bitonic_status_string(status)})")


class bitonic_plan(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tile_log2", ctypes.c_int),
                ("fuse", ctypes.c_int), ("merge_blocks_per_cu", ctypes.c_int)]


_lib = None


def load() -> ctypes.CDLL:
    """The HIP library.  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
            "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sig = {
        "bitonic_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "bitonic_version": ([], ctypes.c_char_p),
        "bitonic_sort_i32": ([vp, ctypes.c_int64, ctypes.c_int, vp], ctypes.c_int),
        "bitonic_sort_plan_i32": ([vp, ctypes.c_int64, ctypes.c_int,
                                   ctypes.POINTER(bitonic_plan), vp], ctypes.c_int),
        "bitonic_sort_segmented_i32": ([vp, vp, ctypes.c_int64, ctypes.c_int, vp],
                                       ctypes.c_int),
        "bitonic_sort_segmented_bounded_i32": ([vp, vp, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_int, vp], ctypes.c_int),
        "bitonic_sort_segmented_noalloc_i32": ([vp, vp, ctypes.c_int64, ctypes.c_int64,
                                               ctypes.c_int, vp], ctypes.c_int),
        "bitonic_segmented_default_bound": ([vp, ctypes.c_int], ctypes.c_int64),
        "bitonic_validation_error": ([ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "bitonic_network_phases_i32": ([vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(bitonic_plan), vp], ctypes.c_int),
        "bitonic_plan_passes": ([ctypes.c_int64, ctypes.POINTER(bitonic_plan)],
                                ctypes.c_int64),
        "bitonic_set_tuning": ([ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
        "bitonic_set_tuning_value": ([ctypes.c_char_p, ctypes.c_int], ctypes.c_int),
        "bitonic_get_tuning_value": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)],
                                     ctypes.c_int),
        "bitonic_graph_capture_sort_i32": ([ctypes.POINTER(vp), vp, ctypes.c_int64, ctypes.c_int,
                                            ctypes.POINTER(bitonic_plan)], ctypes.c_int),
        "bitonic_graph_capture_segmented_i32": ([ctypes.POINTER(vp), vp, vp, ctypes.c_int64,
                                                 ctypes.c_int64, ctypes.c_int], ctypes.c_int),
        "bitonic_graph_launch": ([vp, vp], ctypes.c_int),
        "bitonic_graph_destroy": ([vp], ctypes.c_int),
        "bitonic_load_tuning": ([ctypes.c_char_p], ctypes.c_int),
        "bitonic_keygen_i32": ([vp, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, vp],
                               ctypes.c_int),
        "bitonic_sort_keys": ([vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp], ctypes.c_int),
        "bitonic_sort_keys64": ([vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp],
                                ctypes.c_int),
        "bitonic_sort_pairs": ([vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, vp],
                               ctypes.c_int),
        "bitonic_sort_wide_plan": ([vp, vp, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(bitonic_plan), vp], ctypes.c_int),
        "bitonic_wide_plan_passes": ([ctypes.c_int64, ctypes.POINTER(bitonic_plan)],
                                     ctypes.c_int64),
        "bitonic_plan_tile_log2": ([ctypes.c_int64, ctypes.POINTER(bitonic_plan)], ctypes.c_int),
        "bitonic_sort_segmented_pairs": ([vp, vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                          ctypes.c_int, vp], ctypes.c_int),
        "bitonic_sort_segmented_keys": ([vp, vp, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                                         ctypes.c_int, vp], ctypes.c_int),
        "bitonic_plan_describe": ([ctypes.c_int64, ctypes.POINTER(bitonic_plan), vp, vp,
                                   ctypes.c_int64], ctypes.c_int64),
        "bitonic_sort_plan_launches_i32": ([vp, ctypes.c_int64, ctypes.c_int,
                                            ctypes.POINTER(bitonic_plan), ctypes.c_int64,
                                            ctypes.c_int64, vp], ctypes.c_int),
        "bitonic_plan_shapes": ([ctypes.c_int64, ctypes.c_int, ctypes.POINTER(bitonic_plan),
                                 vp, ctypes.c_int64], ctypes.c_int64),
        "bitonic_sort_plan_events_i32": ([vp, ctypes.c_int64, ctypes.c_int,
                                          ctypes.POINTER(bitonic_plan), vp, ctypes.c_int64,
                                          vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def header_functions(path: str = HEADER) -> list[str]:
    """Names of the functions include/bitonic.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bitonic_[a-z0-9_]+)\s*\(", text)))


def _check(fn: str, rc: int) -> None:
    if rc != 0:
        raise BitonicError(fn, rc)


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _keys_ptr(keys, dtype_name: str = "int32"):
    import torch
    want = torch.int32 if dtype_name == "int32" else torch.int64
    if not isinstance(keys, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU")
    if keys.dtype != want or not keys.is_cuda or not keys.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} tensor on the GPU, got "
                         f"{keys.dtype} on {keys.device} (contiguous={keys.is_contiguous()})")
    return keys.data_ptr() if keys.numel() else None


KEY_TYPES = {"int32": 0, "uint32": 1, "float32": 2, "int64": 3, "uint64": 4, "float64": 5}


def _key_type(keys, key_type) -> int:
    import torch
    if key_type is not None:
        return KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
    by_dtype = {torch.int32: 0, torch.float32: 2}
    if hasattr(torch, "uint32"):
        by_dtype[torch.uint32] = 1
    if keys.dtype not in by_dtype:
        raise ValueError(f"no 32-bit key type for dtype {keys.dtype}")
    return by_dtype[keys.dtype]


def _any32_ptr(keys):
    import torch
    if not isinstance(keys, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU")
    if keys.element_size() != 4 or not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("expected a contiguous tensor of 4-byte keys on the GPU")
    return keys.data_ptr() if keys.numel() else None


def _plan(plan) -> bitonic_plan | None:
    if plan is None:
        return None
    if isinstance(plan, bitonic_plan):
        return plan
    if isinstance(plan, str):
        plan = (plan,)
    kind = plan[0]
    tile = plan[1] if len(plan) > 1 else 0
    fuse = plan[2] if len(plan) > 2 else 0
    bpc = plan[3] if len(plan) > 3 else 0
    return bitonic_plan(PLAN_KINDS[kind] if isinstance(kind, str) else int(kind),
                        int(tile), int(fuse), int(bpc))


def _plan_ref(p):
    return ctypes.byref(p) if p is not None else None


def bitonic_status_string(status: int) -> str:
    return load().bitonic_status_string(int(status)).decode()


def bitonic_version() -> str:
    return load().bitonic_version().decode()


def bitonic_sort_i32(keys, ascending: bool = True, stream=None) -> None:
    """Sort a contiguous int32 GPU tensor in place (asynchronous)."""
    ptr = _keys_ptr(keys)
    _check("bitonic_sort_i32",
           load().bitonic_sort_i32(ptr, keys.numel(), int(bool(ascending)), _stream(stream)))


def bitonic_sort_keys(keys, ascending: bool = True, key_type=None, stream=None) -> None:
    """Sort 4-byte keys in place: int32, uint32 or float32 (IEEE totalOrder),
    taken from the tensor's dtype or given as key_type ("int32", "uint32",
    "float32"; an int32 tensor may hold the bit patterns of another type)."""
    ptr = _any32_ptr(keys)
    _check("bitonic_sort_keys",
           load().bitonic_sort_keys(ptr, keys.numel(), _key_type(keys, key_type),
                                    int(bool(ascending)), _stream(stream)))


def _key_type64(keys, key_type) -> int:
    import torch
    if key_type is not None:
        return KEY_TYPES[key_type] if isinstance(key_type, str) else int(key_type)
    by_dtype = {torch.int64: 3, torch.float64: 5}
    if hasattr(torch, "uint64"):
        by_dtype[torch.uint64] = 4
    if keys.dtype not in by_dtype:
        raise ValueError(f"no 64-bit key type for dtype {keys.dtype}")
    return by_dtype[keys.dtype]


def _any64_ptr(keys):
    import torch
    if not isinstance(keys, torch.Tensor):
        raise TypeError("expected a torch tensor on the GPU")
    if keys.element_size() != 8 or not keys.is_cuda or not keys.is_contiguous():
        raise ValueError("expected a contiguous tensor of 8-byte keys on the GPU")
    return keys.data_ptr() if keys.numel() else None


def bitonic_sort_keys64(keys, ascending: bool = True, key_type=None, stream=None) -> None:
    """Sort 8-byte keys in place: int64, uint64 or float64 (IEEE totalOrder),
    from the tensor's dtype or key_type ("int64", "uint64", "float64"; an
    int64 tensor may hold the bit patterns of another type)."""
    ptr = _any64_ptr(keys)
    _check("bitonic_sort_keys64",
           load().bitonic_sort_keys64(ptr, keys.numel(), _key_type64(keys, key_type),
                                      int(bool(ascending)), _stream(stream)))


def _pair_ptrs(keys, values):
    import torch
    kp = _any32_ptr(keys)
    if not isinstance(values, torch.Tensor) or values.dtype != torch.int32 or \
            not values.is_cuda or not values.is_contiguous():
        raise ValueError("values must be a contiguous int32 tensor on the GPU")
    if values.numel() != keys.numel():
        raise ValueError("keys and values differ in length")
    return kp, (values.data_ptr() if values.numel() else None)


def bitonic_sort_pairs(keys, values, ascending: bool = True, key_type=None, stream=None) -> None:
    """Sort (key, value) pairs in place by key, equal keys by value ascending
    (with values 0..n-1: a stable argsort).  keys: 4-byte keys (int32,
    uint32 or float32, from the dtype or key_type); values: int32."""
    kp, vp_ = _pair_ptrs(keys, values)
    _check("bitonic_sort_pairs",
           load().bitonic_sort_pairs(kp, vp_, keys.numel(), _key_type(keys, key_type),
                                     int(bool(ascending)), _stream(stream)))


def bitonic_sort_wide_plan(keys, values=None, ascending: bool = True, key_type=None,
                           plan=None, stream=None) -> None:
    """An 8-byte sort (values None: 8-byte keys; else pairs) with an explicit
    plan ("optimized", tile_log2 11..13, fuse 1..6)."""
    p = _plan(plan)
    if values is None:
        ptr, vptr, kt = _any64_ptr(keys), None, _key_type64(keys, key_type)
    else:
        (ptr, vptr), kt = _pair_ptrs(keys, values), _key_type(keys, key_type)
    _check("bitonic_sort_wide_plan",
           load().bitonic_sort_wide_plan(ptr, vptr, keys.numel(), kt, int(bool(ascending)),
                                         _plan_ref(p), _stream(stream)))


def bitonic_wide_plan_passes(n: int, plan=None) -> int:
    p = _plan(plan)
    return int(load().bitonic_wide_plan_passes(int(n), _plan_ref(p)))


def bitonic_sort_segmented_pairs(keys, values, offsets, ascending: bool = True, key_type=None,
                                 max_seg_len: int | None = None, stream=None) -> None:
    """Sort (key, value) pairs per CSR segment: by key, equal keys by value
    (values 0..len-1 per segment give a stable per-segment argsort)."""
    kp, vptr = _pair_ptrs(keys, values)
    op = _keys_ptr(offsets, "int64")
    nseg = max(offsets.numel() - 1, 0)
    _check("bitonic_sort_segmented_pairs",
           load().bitonic_sort_segmented_pairs(kp, vptr, op, nseg, int(max_seg_len or 0),
                                               _key_type(keys, key_type), int(bool(ascending)),
                                               _stream(stream)))


def bitonic_sort_segmented_keys(keys, offsets, ascending: bool = True, key_type=None,
                                max_seg_len: int = 0, stream=None) -> None:
    """Per-segment sort of keys of any type: 4-byte (int32, uint32, float32)
    or 8-byte (int64, uint64, float64), from the dtype or key_type."""
    if keys.element_size() == 8:
        kp, kt = _any64_ptr(keys), _key_type64(keys, key_type)
        op = _keys_ptr(offsets, "int64")
        _check("bitonic_sort_segmented_keys",
               load().bitonic_sort_segmented_keys(kp, op, max(offsets.numel() - 1, 0),
                                                  int(max_seg_len), kt, int(bool(ascending)),
                                                  _stream(stream)))
        return
    kp = _any32_ptr(keys)
    op = _keys_ptr(offsets, "int64")
    _check("bitonic_sort_segmented_keys",
           load().bitonic_sort_segmented_keys(kp, op, max(offsets.numel() - 1, 0),
                                              int(max_seg_len), _key_type(keys, key_type),
                                              int(bool(ascending)), _stream(stream)))


def bitonic_sort_plan_i32(keys, ascending: bool = True, plan=None, stream=None) -> None:
    """bitonic_sort_i32 with an explicit plan: ("basic"|"semi"|"optimized",
    tile_log2, fuse)."""
    ptr = _keys_ptr(keys)
    p = _plan(plan)
    _check("bitonic_sort_plan_i32",
           load().bitonic_sort_plan_i32(ptr, keys.numel(), int(bool(ascending)), _plan_ref(p),
                                        _stream(stream)))


def bitonic_network_phases_i32(keys, last_phase: int, ascending: bool = True, plan=None,
                               stream=None) -> None:
    ptr = _keys_ptr(keys)
    p = _plan(plan)
    _check("bitonic_network_phases_i32",
           load().bitonic_network_phases_i32(ptr, keys.numel(), int(bool(ascending)),
                                             int(last_phase), _plan_ref(p), _stream(stream)))


def bitonic_sort_segmented_i32(keys, offsets, ascending: bool = True, stream=None,
                               max_seg_len: int | None = None) -> None:
    """Sort every CSR segment of ``keys`` (int64 ``offsets`` on the GPU)."""
    kp = _keys_ptr(keys)
    op = _keys_ptr(offsets, "int64")
    nseg = max(offsets.numel() - 1, 0)
    if max_seg_len is None:
        _check("bitonic_sort_segmented_i32",
               load().bitonic_sort_segmented_i32(kp, op, nseg, int(bool(ascending)),
                                                 _stream(stream)))
    else:
        _check("bitonic_sort_segmented_bounded_i32",
               load().bitonic_sort_segmented_bounded_i32(kp, op, nseg, int(max_seg_len),
                                                         int(bool(ascending)),
                                                         _stream(stream)))


def bitonic_sort_segmented_noalloc_i32(keys, offsets, max_seg_len: int, ascending: bool = True,
                                       stream=None) -> None:
    """The allocation-free segmented sort (a library-owned device array as
    scratch; at most 2^18 - 1 segments; calls overlapping on one GPU race)."""
    kp = _keys_ptr(keys)
    op = _keys_ptr(offsets, "int64")
    _check("bitonic_sort_segmented_noalloc_i32",
           load().bitonic_sort_segmented_noalloc_i32(kp, op, max(offsets.numel() - 1, 0),
                                                     int(max_seg_len), int(bool(ascending)),
                                                     _stream(stream)))


def bitonic_segmented_default_bound(keys) -> int:
    """The segment-length bound the segmented sorts take for ``keys`` when
    no bound is given (end of the keys' device allocation, at most 2^31)."""
    return int(load().bitonic_segmented_default_bound(keys.data_ptr(), keys.element_size()))


def bitonic_validation_error() -> int:
    """The first segment-table error recorded by a validated segmented sort
    since the last call (0: none); waits for the device, clears the record."""
    c = ctypes.c_int32()
    _check("bitonic_validation_error", load().bitonic_validation_error(ctypes.byref(c)))
    return int(c.value)


def bitonic_plan_tile_log2(n: int, plan=None) -> int:
    p = _plan(plan)
    return int(load().bitonic_plan_tile_log2(int(n), _plan_ref(p)))


def bitonic_plan_passes(n: int, plan=None) -> int:
    p = _plan(plan)
    return int(load().bitonic_plan_passes(int(n), _plan_ref(p)))


LAUNCH_KINDS = {1: "tile_sort", 2: "global_pass", 3: "tile_merge", 4: "lds_network",
                5: "step"}


def bitonic_plan_describe(n: int, plan=None) -> list[tuple[str, int]]:
    """[(launch kind, fused steps)] for every launch of the plan for n keys."""
    import numpy as np
    p = _plan(plan)
    m = int(load().bitonic_plan_describe(int(n), _plan_ref(p), None, None, 0))
    if m < 0:
        raise BitonicError("bitonic_plan_describe", m)
    kinds = np.zeros(max(m, 1), np.int32)
    fuse = np.zeros(max(m, 1), np.int32)
    load().bitonic_plan_describe(int(n), _plan_ref(p), kinds.ctypes.data, fuse.ctypes.data, m)
    return [(LAUNCH_KINDS[int(k)], int(f)) for k, f in zip(kinds[:m], fuse[:m])]


class bitonic_launch_shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fuse", ctypes.c_int32), ("q", ctypes.c_int32),
                ("mirror", ctypes.c_int32), ("elem_bytes", ctypes.c_int32),
                ("offset_bits", ctypes.c_int32)]


LAYOUTS = {"keys32": 0, "keys32_unaligned": 1, "keys64": 2, "pairs": 3, "seg_keys32": 4,
           "seg_pairs": 5, "seg_keys64": 6}
LAUNCH_KINDS.update({6: "seg_prep", 7: "seg_small"})


def bitonic_plan_shapes(n: int, layout: str = "keys32", plan=None) -> list[dict]:
    """The shape of every launch of a sort of n elements (bitonic_plan_shapes):
    [{kind, fuse, q, mirror, elem_bytes, offset_bits}]."""
    p = _plan(plan)
    lay = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
    m = int(load().bitonic_plan_shapes(int(n), lay, _plan_ref(p), None, 0))
    if m < 0:
        raise BitonicError("bitonic_plan_shapes", m)
    arr = (bitonic_launch_shape * max(m, 1))()
    load().bitonic_plan_shapes(int(n), lay, _plan_ref(p), ctypes.cast(arr, ctypes.c_void_p), m)
    return [{"kind": LAUNCH_KINDS[a.kind], "fuse": a.fuse, "q": a.q, "mirror": a.mirror,
             "elem_bytes": a.elem_bytes, "offset_bits": a.offset_bits} for a in arr[:m]]


class HipEvents:
    """A set of HIP events (created through the HIP runtime) for timing."""

    def __init__(self, count: int):
        self.rt = ctypes.CDLL("libamdhip64.so")
        self.rt.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self.rt.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float),
                                                ctypes.c_void_p, ctypes.c_void_p]
        self.rt.hipEventSynchronize.argtypes = [ctypes.c_void_p]
        self.rt.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.ev = (ctypes.c_void_p * count)()
        for i in range(count):
            e = ctypes.c_void_p()
            if self.rt.hipEventCreate(ctypes.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev[i] = e
        self.count = count

    def elapsed_ms(self, a: int, b: int) -> float:
        self.rt.hipEventSynchronize(self.ev[b])
        ms = ctypes.c_float()
        if self.rt.hipEventElapsedTime(ctypes.byref(ms), self.ev[a], self.ev[b]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for i in range(self.count):
            self.rt.hipEventDestroy(self.ev[i])
        self.count = 0


def bitonic_sort_plan_events_i32(keys, events: HipEvents, ascending: bool = True, plan=None,
                                 stream=None) -> None:
    """Sort recording events[0] before and events[i + 1] after launch i."""
    ptr = _keys_ptr(keys)
    p = _plan(plan)
    _check("bitonic_sort_plan_events_i32",
           load().bitonic_sort_plan_events_i32(ptr, keys.numel(), int(bool(ascending)),
                                               _plan_ref(p), ctypes.cast(events.ev, ctypes.c_void_p),
                                               events.count, _stream(stream)))


def bitonic_sort_plan_launches_i32(keys, first: int, count: int, ascending: bool = True,
                                   plan=None, stream=None) -> None:
    """Enqueue launches [first, first + count) of the plan only (timing)."""
    ptr = _keys_ptr(keys)
    p = _plan(plan)
    _check("bitonic_sort_plan_launches_i32",
           load().bitonic_sort_plan_launches_i32(ptr, keys.numel(), int(bool(ascending)),
                                                 _plan_ref(p), int(first), int(count),
                                                 _stream(stream)))


def bitonic_set_tuning(tile_log2: int = 0, fuse: int = 0, merge_blocks_per_cu: int = 0) -> None:
    _check("bitonic_set_tuning", load().bitonic_set_tuning(int(tile_log2), int(fuse),
                                                           int(merge_blocks_per_cu)))


def bitonic_set_tuning_value(key: str, value: int) -> None:
    _check("bitonic_set_tuning_value", load().bitonic_set_tuning_value(key.encode(), int(value)))


def bitonic_get_tuning_value(key: str) -> int:
    v = ctypes.c_int()
    _check("bitonic_get_tuning_value", load().bitonic_get_tuning_value(key.encode(),
                                                                       ctypes.byref(v)))
    return int(v.value)


class BitonicGraph:
    """A captured sort (bitonic_graph_*): replay with launch(), free with
    close() once every replay has finished."""

    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream=None) -> None:
        _check("bitonic_graph_launch", load().bitonic_graph_launch(self.handle, _stream(stream)))

    def close(self) -> None:
        if self.handle:
            load().bitonic_graph_destroy(self.handle)
            self.handle = None


def bitonic_graph_capture_sort_i32(keys, ascending: bool = True, plan=None) -> BitonicGraph:
    ptr = _keys_ptr(keys)
    p = _plan(plan)
    h = ctypes.c_void_p()
    _check("bitonic_graph_capture_sort_i32",
           load().bitonic_graph_capture_sort_i32(ctypes.byref(h), ptr, keys.numel(),
                                                 int(bool(ascending)), _plan_ref(p)))
    return BitonicGraph(h)


def bitonic_graph_capture_segmented_i32(keys, offsets, max_seg_len: int,
                                        ascending: bool = True) -> BitonicGraph:
    kp = _keys_ptr(keys)
    op = _keys_ptr(offsets, "int64")
    h = ctypes.c_void_p()
    _check("bitonic_graph_capture_segmented_i32",
           load().bitonic_graph_capture_segmented_i32(ctypes.byref(h), kp, op,
                                                      max(offsets.numel() - 1, 0),
                                                      int(max_seg_len), int(bool(ascending))))
    return BitonicGraph(h)


def bitonic_load_tuning(path: str) -> None:
    _check("bitonic_load_tuning", load().bitonic_load_tuning(path.encode()))


def bitonic_keygen_i32(out, seed: int, start: int = 0, stream=None) -> None:
    """Fill an int32 GPU tensor with the SplitMix64 key stream ``seed``."""
    ptr = _keys_ptr(out)
    _check("bitonic_keygen_i32",
           load().bitonic_keygen_i32(ptr, out.numel(), int(seed) & (2**64 - 1), int(start),
                                     _stream(stream)))
