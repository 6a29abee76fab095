"""Autotuner for the bitonic sort library.

python -m paper_1506_01446_amd.autotune [--n 16777216] [--out tuning.txt]

Searches, on the GPU, the plan parameters that do not change the result:
  tile_log2            keys per on-chip tile (2^12 .. 2^15)
  fuse                 long-stride steps fused per HBM pass (5 .. 8)
  merge_blocks_per_cu  tile-merge workgroups per compute unit (-1: one tile each)
for the single-array sort of n keys, and
  seg_blocks_per_cu    workgroups per compute unit of the persistent
                       small-segment kernel
  seg_pass_blocks_per_cu  workgroups per compute unit of the big-segment
                       passes
on the batched segmented workload.  Every candidate is timed with HIP events
over fresh copies of the same seeded input (median of several runs) and its
output checked sorted; the fastest are written as "<name> <value>" lines that
bitonic_load_tuning reads.
"""
from __future__ import annotations

import argparse
import itertools
import json
import statistics
import sys

from . import binding as B
from . import workloads as W


def _time_plain(torch, src, plan, reps: int) -> float:
    ev = B.HipEvents(2)
    rt = ev.rt
    rt.hipEventRecord.argtypes = [B.ctypes.c_void_p, B.ctypes.c_void_p]
    st = torch.cuda.current_stream().cuda_stream
    times = []
    buf = src.clone()
    B.bitonic_sort_plan_i32(buf, True, plan)  # warm
    for _ in range(reps):
        buf.copy_(src)
        torch.cuda.synchronize()
        rt.hipEventRecord(ev.ev[0], st)
        B.bitonic_sort_plan_i32(buf, True, plan)
        rt.hipEventRecord(ev.ev[1], st)
        torch.cuda.synchronize()
        times.append(ev.elapsed_ms(0, 1))
    ok = bool((buf[1:] >= buf[:-1]).all().item())
    ev.close()
    if not ok:
        raise RuntimeError(f"plan {plan} produced unsorted output")
    return statistics.median(times)


def _time_segmented(torch, keys, offs, max_len, reps: int) -> float:
    ev = B.HipEvents(2)
    rt = ev.rt
    rt.hipEventRecord.argtypes = [B.ctypes.c_void_p, B.ctypes.c_void_p]
    st = torch.cuda.current_stream().cuda_stream
    buf = keys.clone()
    B.bitonic_sort_segmented_i32(buf, offs, True, max_seg_len=max_len)
    times = []
    for _ in range(reps):
        buf.copy_(keys)
        torch.cuda.synchronize()
        rt.hipEventRecord(ev.ev[0], st)
        B.bitonic_sort_segmented_i32(buf, offs, True, max_seg_len=max_len)
        rt.hipEventRecord(ev.ev[1], st)
        torch.cuda.synchronize()
        times.append(ev.elapsed_ms(0, 1))
    ev.close()
    return statistics.median(times)


def tune(n: int = 1 << 24, reps: int = 5, quick: bool = False, log=print) -> dict:
    import torch
    B.load()
    src = torch.from_numpy(W.uniform_i32(W.SEED_BASE + 2, n)).cuda()
    tiles = (14,) if quick else (12, 13, 14, 15)
    fuses = (7, 8) if quick else (5, 6, 7, 8)
    merges = (2,) if quick else (-1, 1, 2, 4)
    results = []
    for t, f, m in itertools.product(tiles, fuses, merges):
        ms = _time_plain(torch, src, ("optimized", t, f, m), reps)
        results.append((ms, t, f, m))
        log(json.dumps({"tile_log2": t, "fuse": f, "merge_blocks_per_cu": m, "ms": round(ms, 4)}))
    results.sort()
    best = results[0]
    keys, off = W.batched_workload()
    kt = torch.from_numpy(keys).cuda()
    ot = torch.from_numpy(off).cuda()
    max_len = int((off[1:] - off[:-1]).max())
    seg = []
    for bpc in ((4,) if quick else (2, 3, 4, 6)):
        B.bitonic_set_tuning_value("seg_blocks_per_cu", bpc)
        ms = _time_segmented(torch, kt, ot, max_len, reps)
        seg.append((ms, bpc))
        log(json.dumps({"seg_blocks_per_cu": bpc, "ms": round(ms, 4)}))
    seg.sort()
    B.bitonic_set_tuning_value("seg_blocks_per_cu", seg[0][1])
    segp = []
    for bpc in ((8,) if quick else (4, 8, 16)):
        B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", bpc)
        ms = _time_segmented(torch, kt, ot, max_len, reps)
        segp.append((ms, bpc))
        log(json.dumps({"seg_pass_blocks_per_cu": bpc, "ms": round(ms, 4)}))
    segp.sort()
    B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", segp[0][1])
    return {"tile_log2": best[1], "fuse": best[2], "merge_blocks_per_cu": best[3],
            "seg_blocks_per_cu": seg[0][1], "seg_pass_blocks_per_cu": segp[0][1],
            "sort_ms": round(best[0], 4), "segmented_ms": round(segp[0][0], 4), "n": n}


def write_tuning(path: str, best: dict) -> None:
    with open(path, "w") as f:
        f.write(f"tile_log2 {best['tile_log2']}\n")
        f.write(f"fuse {best['fuse']}\n")
        f.write(f"merge_blocks_per_cu {best['merge_blocks_per_cu']}\n")
        f.write(f"seg_blocks_per_cu {best['seg_blocks_per_cu']}\n")
        if "seg_pass_blocks_per_cu" in best:
            f.write(f"seg_pass_blocks_per_cu {best['seg_pass_blocks_per_cu']}\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=1 << 24)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default="tuning.txt")
    a = ap.parse_args(argv)
    best = tune(a.n, a.reps, a.quick, log=lambda s: print(s, file=sys.stderr, flush=True))
    write_tuning(a.out, best)
    B.bitonic_load_tuning(a.out)
    print(json.dumps(best))
    return 0


if __name__ == "__main__":
    sys.exit(main())
