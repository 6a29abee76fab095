"""Autotuner for the bitonic sort library.

python -m paper_1506_01446_amd.autotune [--buckets 16,18,20,22,24,26,28]
        [--reps 5] [--out paper_1506_01446_amd/tuning/mi355x.txt]
        [--log <full log>] [--summary profiles/autotune_mi355x.txt]

Searches, on the GPU, the plan parameters that do not change the result
(the paper leaves the shared-memory tile and the register fusion depth open,
sections 4.1 and 4.2):
  per size bucket k (n = 2^k keys, single-array 4-byte sort)
    tile_log2            keys per on-chip tile (2^12 .. 2^15)
    fuse                 long-stride steps fused per HBM pass (6 .. 10)
    merge_blocks_per_cu  tile-merge workgroups per compute unit (-1: one
                         tile each)
  sort_tile_log2@k       a tile sort of larger tiles than the merges' (one
                         launch fewer, a longer tile sort), per bucket from
                         2^20 up where it is 0.3 % faster
  lane_pass              how passes of eight to ten steps split columns
                         over lanes or waves (7, 8 or 9), by the tuned plans
                         of the buckets from 2^22 up (their times relative to
                         each bucket's best mode, averaged), then per bucket
                         ("lane_pass@k") where another mode is 1 % faster
  phase_blocks_per_cu    workgroups of the tile phase (phase t+1 in one
                         launch) per compute unit, -1, 1, 2 or 4, by the
                         tuned plans from 2^20 up (relative times, averaged)
  segmented sort (the 8192-segment batched workload, and a table of 64
  segments of the serving workload's lengths, 2^8 .. 2^22 keys)
    seg_blocks_per_cu       small-segment kernel workgroups per compute unit
    seg_pass_blocks_per_cu  big-segment pass workgroups per compute unit
    seg_fuse                steps per big-segment pass (3 .. 5)
  8-byte sorts (int64 keys and int32 (key, value) pairs at n = 2^24, by
  their summed time)
    wide_tile_log2, wide_fuse
Every candidate is timed with HIP events over fresh copies of the same seeded
input (median of `reps` runs) and its output checked sorted.  The winners are
written as "<name> <value>" lines (bucket entries as "name@k", only where
the tuned plan beats the built-in one by 1 % or more) under a "cus <count>"
line, which bitonic_load_tuning reads; every timing goes to the log, one JSON
object per line, and a short summary (per bucket the five fastest plans and
the winner against the built-in plan; the segmented and 8-byte timings in
full) to --summary.
"""
from __future__ import annotations

import argparse
import datetime
import itertools
import json
import os
import statistics
import sys

from . import binding as B
from . import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning", "mi355x.txt")


def _events(torch):
    ev = B.HipEvents(2)
    rt = ev.rt
    rt.hipEventRecord.argtypes = [B.ctypes.c_void_p, B.ctypes.c_void_p]
    return ev, rt, torch.cuda.current_stream().cuda_stream


def _median_ms(torch, reset, run, reps: int) -> float:
    ev, rt, st = _events(torch)
    reset()
    run()
    times = []
    for _ in range(reps):
        reset()
        torch.cuda.synchronize()
        rt.hipEventRecord(ev.ev[0], st)
        run()
        rt.hipEventRecord(ev.ev[1], st)
        torch.cuda.synchronize()
        times.append(ev.elapsed_ms(0, 1))
    ev.close()
    return statistics.median(times)


def _time_plain(torch, src, buf, plan, reps: int) -> float:
    ms = _median_ms(torch, lambda: buf.copy_(src),
                    lambda: B.bitonic_sort_plan_i32(buf, True, plan), reps)
    if not bool((buf[1:] >= buf[:-1]).all().item()):
        raise RuntimeError(f"plan {plan} produced unsorted output")
    return ms


def _segment_tables(torch):
    """The batched workload and a serving-sized table, on the device."""
    keys, off = W.batched_workload()
    lens = W.segment_lengths(W.SEED_BASE + 40, 64, 14.0)
    lens = (lens * 256).clip(256, 1 << 22)            # 2^8 .. 2^22 keys
    off2 = W.offsets_from_lengths(lens)
    keys2 = W.uniform_i32(W.SEED_BASE + 41, int(off2[-1]))
    out = []
    for k, o in ((keys, off), (keys2, off2)):
        out.append((torch.from_numpy(k).cuda(), torch.from_numpy(o).cuda(),
                    int((o[1:] - o[:-1]).max())))
    return out


def _time_segmented(torch, tables, reps: int) -> float:
    total = 0.0
    for kt, ot, mx in tables:
        buf = kt.clone()
        total += _median_ms(torch, lambda: buf.copy_(kt),
                            lambda: B.bitonic_sort_segmented_i32(buf, ot, True, max_seg_len=mx),
                            reps)
    return total


def tune(buckets=(16, 18, 20, 22, 24, 26, 28), reps: int = 5, quick: bool = False,
         log=print) -> dict:
    import torch
    B.load()
    best = {"cus": torch.cuda.get_device_properties(0).multi_processor_count,
            "device": torch.cuda.get_device_name(0), "buckets": {}}
    tiles = (13, 14) if quick else (12, 13, 14, 15)
    fuses = (8, 10) if quick else (6, 7, 8, 9, 10)
    merges = (2,) if quick else (-1, 1, 2, 4)
    for k in buckets:
        n = 1 << k
        src = torch.empty(n, dtype=torch.int32, device="cuda")
        B.bitonic_keygen_i32(src, W.SEED_BASE + k)
        buf = torch.empty_like(src)
        default_ms = _time_plain(torch, src, buf, None, reps)
        rows = []
        for t, f, m in itertools.product(tiles, fuses, merges):
            if t > k:
                continue
            ms = _time_plain(torch, src, buf, ("optimized", t, f, m), reps)
            rows.append((ms, t, f, m))
            log(json.dumps({"bucket": k, "tile_log2": t, "fuse": f, "merge_blocks_per_cu": m,
                            "ms": round(ms, 4)}))
        rows.sort()
        ms, t, f, m = rows[0]
        best["buckets"][k] = {"tile_log2": t, "fuse": f, "merge_blocks_per_cu": m,
                              "ms": round(ms, 4), "default_ms": round(default_ms, 4)}
        log(json.dumps({"bucket": k, "best": best["buckets"][k]}))
        del src, buf
    def bucket_times(lo):
        times = {}
        for k, e in best["buckets"].items():
            if k < lo:
                continue
            src = torch.empty(1 << k, dtype=torch.int32, device="cuda")
            B.bitonic_keygen_i32(src, W.SEED_BASE + k)
            buf = torch.empty_like(src)
            times[k] = _time_plain(torch, src, buf, ("optimized", e["tile_log2"], e["fuse"],
                                                     e["merge_blocks_per_cu"]), reps)
            del src, buf
        return times

    def pick_global(name, values, lo):
        """The value of a global knob whose tuned plans of the buckets from
        2^lo up are fastest on average relative to each bucket's best value
        (every bucket weighs the same, not the largest's milliseconds)."""
        times = {}
        for v in values:
            B.bitonic_set_tuning_value(name, v)
            times[v] = bucket_times(lo)
        rel = {v: statistics.mean(times[v][k] / min(times[u][k] for u in values)
                                  for k in times[v]) for v in values}
        for v in values:
            log(json.dumps({name: v, f"ms_buckets_{lo}_up": round(sum(times[v].values()), 4),
                            "mean_over_best": round(rel[v], 5)}))
        v = min(values, key=rel.get)
        B.bitonic_set_tuning_value(name, v)
        return v

    best["phase_blocks_per_cu"] = pick_global("phase_blocks_per_cu",
                                              (1,) if quick else (-1, 1, 2, 4), 20)
    best["lane_pass"] = pick_global("lane_pass", (7, 8), 22)
    # and per bucket from 2^22 up: a bucket entry where another mode beats
    # the global one by 1 % or more
    for k, e in best["buckets"].items():
        if k < 22 or quick:
            continue
        src = torch.empty(1 << k, dtype=torch.int32, device="cuda")
        B.bitonic_keygen_i32(src, W.SEED_BASE + k)
        buf = torch.empty_like(src)
        plan = ("optimized", e["tile_log2"], e["fuse"], e["merge_blocks_per_cu"])
        times = {}
        for mode in (7, 8, 9):
            B.bitonic_set_tuning_value(f"lane_pass@{k}", mode)
            times[mode] = _time_plain(torch, src, buf, plan, reps)
            log(json.dumps({"bucket": k, "lane_pass": mode, "ms": round(times[mode], 4)}))
        B.bitonic_set_tuning_value(f"lane_pass@{k}", 0)
        mode = min(times, key=times.get)
        if mode != best["lane_pass"] and times[mode] < 0.99 * times[best["lane_pass"]]:
            e["lane_pass"] = mode
            B.bitonic_set_tuning_value(f"lane_pass@{k}", mode)
        del src, buf
    # and per bucket from 2^20 up: a tile sort of larger tiles than the
    # merges' ("sort_tile_log2@k"), which saves a launch for a longer tile
    # sort, where it beats the bucket's plan by 0.3 % or more (medians of
    # four times as many sorts: the difference is a fraction of a percent)
    for k, e in best["buckets"].items():
        if k < 20 or quick or e["tile_log2"] >= 15:
            continue
        src = torch.empty(1 << k, dtype=torch.int32, device="cuda")
        B.bitonic_keygen_i32(src, W.SEED_BASE + k)
        buf = torch.empty_like(src)
        plan = ("optimized", e["tile_log2"], e["fuse"], e["merge_blocks_per_cu"])
        times = {}
        for st in (0,) + tuple(range(e["tile_log2"] + 1, 16)):
            B.bitonic_set_tuning_value(f"sort_tile_log2@{k}", st)
            times[st] = _time_plain(torch, src, buf, plan, 4 * reps)
            log(json.dumps({"bucket": k, "sort_tile_log2": st, "ms": round(times[st], 4)}))
        st = min(times, key=times.get)
        if st and times[st] < 0.997 * times[0]:
            e["sort_tile_log2"] = st
        B.bitonic_set_tuning_value(f"sort_tile_log2@{k}", e.get("sort_tile_log2", 0))
        del src, buf
    tables = _segment_tables(torch)
    seg = []
    for bpc in ((4,) if quick else (2, 3, 4, 6, 8)):
        B.bitonic_set_tuning_value("seg_blocks_per_cu", bpc)
        ms = _time_segmented(torch, tables[:1], reps)
        seg.append((ms, bpc))
        log(json.dumps({"seg_blocks_per_cu": bpc, "ms": round(ms, 4)}))
    seg.sort()
    B.bitonic_set_tuning_value("seg_blocks_per_cu", seg[0][1])
    segp = []
    for bpc, sf in itertools.product((8,) if quick else (4, 8, 16), (5,) if quick else (3, 4, 5)):
        B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", bpc)
        B.bitonic_set_tuning_value("seg_fuse", sf)
        ms = _time_segmented(torch, tables, reps)
        segp.append((ms, bpc, sf))
        log(json.dumps({"seg_pass_blocks_per_cu": bpc, "seg_fuse": sf, "ms_both_tables": round(ms, 4)}))
    segp.sort()
    B.bitonic_set_tuning_value("seg_pass_blocks_per_cu", segp[0][1])
    B.bitonic_set_tuning_value("seg_fuse", segp[0][2])
    best.update({"seg_blocks_per_cu": seg[0][1], "seg_pass_blocks_per_cu": segp[0][1],
                 "seg_fuse": segp[0][2], "segmented_ms": round(segp[0][0], 4)})
    del tables
    n = 1 << 24
    k64 = torch.from_numpy(W.uniform_i64(W.SEED_BASE + 2, n)).cuda()
    buf = torch.empty_like(k64)
    k32 = torch.from_numpy(W.uniform_i32(W.SEED_BASE + 2, n)).cuda()
    v32 = torch.arange(n, dtype=torch.int32, device="cuda")
    kbuf, vbuf = torch.empty_like(k32), torch.empty_like(v32)

    def reset_pairs():
        kbuf.copy_(k32)
        vbuf.copy_(v32)

    wide = []
    for t, f in itertools.product((13,) if quick else (11, 12, 13), (8,) if quick else (5, 6, 7, 8)):
        plan = ("optimized", t, f)
        ms = _median_ms(torch, lambda: buf.copy_(k64),
                        lambda: B.bitonic_sort_wide_plan(buf, None, True, "int64", plan), reps)
        if not bool((buf[1:] >= buf[:-1]).all().item()):
            raise RuntimeError(f"8-byte plan {plan} produced unsorted output")
        ms_pairs = _median_ms(torch, reset_pairs,
                              lambda: B.bitonic_sort_wide_plan(kbuf, vbuf, True, "int32", plan),
                              reps)
        if not bool((kbuf[1:] >= kbuf[:-1]).all().item()):
            raise RuntimeError(f"8-byte plan {plan} produced unsorted pairs")
        # int64 keys and (key, value) pairs weigh the same
        wide.append((ms + ms_pairs, t, f))
        log(json.dumps({"wide_tile_log2": t, "wide_fuse": f, "ms": round(ms, 4),
                        "ms_pairs": round(ms_pairs, 4)}))
    wide.sort()
    best.update({"wide_tile_log2": wide[0][1], "wide_fuse": wide[0][2],
                 "wide_ms": round(wide[0][0], 4)})
    return best


def write_tuning(path: str, best: dict, command: str = "") -> None:
    """The tuning file: global values, then per-bucket entries; with "cus"
    when known.  Accepts the autotuner's result or a plain dict of global
    values."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        if "device" in best:
            f.write(f"# bitonic sort plan table, autotuned on {best['device']} "
                    f"({best['cus']} compute units), {datetime.date.today()}\n")
        if command:
            f.write(f"# command: {command}\n")
        if "cus" in best:
            f.write(f"cus {best['cus']}\n")
        for name in ("tile_log2", "fuse", "merge_blocks_per_cu", "lane_pass", "phase_blocks_per_cu",
                     "seg_blocks_per_cu",
                     "seg_pass_blocks_per_cu", "seg_fuse", "wide_tile_log2", "wide_fuse"):
            if name in best:
                f.write(f"{name} {best[name]}\n")
        for k, e in sorted(best.get("buckets", {}).items()):
            f.write(f"# n = 2^{k}: {e['ms']} ms tuned, {e['default_ms']} ms with the built-in plan\n")
            # a bucket's plan entries only where they pay, or where a lane
            # mode or tile-sort tile was timed with that plan for the bucket
            if e["ms"] < 0.99 * e["default_ms"] or "lane_pass" in e or "sort_tile_log2" in e:
                for name in ("tile_log2", "fuse", "merge_blocks_per_cu"):
                    f.write(f"{name}@{k} {e[name]}\n")
            if "lane_pass" in e:
                f.write(f"lane_pass@{k} {e['lane_pass']}\n")
            if "sort_tile_log2" in e:
                f.write(f"sort_tile_log2@{k} {e['sort_tile_log2']}\n")


def write_summary(path: str, rows: list, command: str) -> None:
    """The condensed timing table: per size bucket the five fastest plans and
    the winner, then every segmented and 8-byte timing."""
    out = ["# autotuner timings (ms, median of --reps runs), one JSON object per line",
           f"# command: {command}",
           "# per size bucket: the five fastest plans of those timed, then the winner",
           "# against the built-in plan; the segmented and 8-byte knobs in full"]
    for k in sorted({r["bucket"] for r in rows if "bucket" in r}):
        cand = sorted((r for r in rows if r.get("bucket") == k and "ms" in r),
                      key=lambda r: r["ms"])
        out.append(f"## n = 2^{k}: {len(cand)} plans timed, slowest {cand[-1]['ms']} ms"
                   if cand else f"## n = 2^{k}")
        out += [json.dumps(r) for r in cand[:5]]
        out += [json.dumps(r) for r in cand[5:] if "sort_tile_log2" in r]
        out += [json.dumps(r) for r in rows if r.get("bucket") == k and "best" in r]
    out.append("## segmented and 8-byte knobs")
    out += [json.dumps(r) for r in rows if "bucket" not in r]
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--buckets", default="16,18,20,22,24,26,28")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--quick", action="store_true")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--log", default="")
    ap.add_argument("--summary", default="")
    a = ap.parse_args(argv)
    buckets = tuple(int(x) for x in a.buckets.split(",") if x)
    command = "python -m paper_1506_01446_amd.autotune " + " ".join(
        argv if argv is not None else sys.argv[1:])
    logf = open(a.log, "w") if a.log else None
    rows = []

    def log(s):
        print(s, file=sys.stderr, flush=True)
        rows.append(json.loads(s))
        if logf:
            logf.write(s + "\n")
            logf.flush()

    if logf:
        logf.write("# autotuner timings (ms, median of --reps runs), one JSON object per line\n")
        logf.write(f"# command: {command}\n")
    best = tune(buckets, a.reps, a.quick, log=log)
    write_tuning(a.out, best, command)
    if a.summary:
        write_summary(a.summary, rows, command)
    B.bitonic_load_tuning(a.out)
    print(json.dumps(best))
    if logf:
        logf.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
