"""Benchmark of the exact-selectivity hot path on one MI355X.

Workload (default): the 300M-row fact table with 8 columns (int32 date over
2557 days, int8 quantity 1-50, int8 discount 0-10, int64 log-normal price with
5 % NULLs, three Zipf(1.1) dictionary-coded string columns of 7 / 25 / 4500
codes, an unreferenced int32 key) and the 6-leaf AND/OR predicate with a
10-code IN-list and a LIKE pre-resolved to a 4500-bit code bitmap.

One step = one pass of the whole path over the resident table: compile the
predicate program, run the fused evaluate + COUNT scan (which also writes the
result mask), compare the count with Algorithm 1's limit maxSize, and
materialise the qualifying row ids in ascending order.  `value` is rows of
the table processed per second by that step.

Prints ONE JSON line.  Kernel times come from HIP events that libsel records
on its own stream around each launch.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published peak
MAX_SELECTIVITY = 0.05    # PUSH_DOWN_MAX_SELECTIVITY used for maxSize


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def cpu_baseline(table, tree, threads):
    """The oracle as it stands, on the machine's host cores, over the same table
    (all rows, row ranges split over `threads` threads)."""
    import oracle
    orc = oracle.Oracle(table)
    t0 = time.perf_counter()
    c = orc.count(tree, threads=threads)
    dt = time.perf_counter() - t0
    return c, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=300_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=50)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (a plain "
                         "copy kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    from paper_1806_08384_amd import sel

    threads = host_threads()
    log(f"generating {args.rows} rows ({threads} threads)")
    t0 = time.perf_counter()
    table = datagen.cfg2(n=args.rows, threads=threads)
    log(f"generated in {time.perf_counter() - t0:.1f}s")
    tree = datagen.cfg2_predicate()

    ctx = sel.Context(0)
    dt = sel.device_table(ctx, table)
    n = table.nrows
    max_rows = sel.max_rows(n, MAX_SELECTIVITY)
    ids = torch.empty(max(1, max_rows), dtype=torch.int32, device="cuda")

    def step():
        prog = ctx.program(dt, tree)
        st, cnt = ctx.pushdown_rowids(dt, prog, max_rows, ids)
        if st != sel.SEL_OK:
            raise RuntimeError(f"push-down status {st}")
        return cnt, prog

    log("warmup")
    cnt = None
    for _ in range(args.warmup):
        cnt, prog = step()
    ctx.enable_timing(True)
    ctx.read_timing(reset=True)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cnt, prog = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms, launches = ctx.read_timing(reset=True)

    bpr = prog.bytes_per_row                       # referenced columns + validity
    ntiles = (n + 2047) // 2048
    mask_bytes = ntiles * 64 * 4
    mask_kernel_bytes = n * bpr + mask_bytes + ntiles * 4
    mask_avg_s = ms[sel.K_MASK] / max(1, launches[sel.K_MASK]) / 1e3
    compact_avg_s = ms[sel.K_COMPACT] / max(1, launches[sel.K_COMPACT]) / 1e3
    scan_avg_s = ms[sel.K_SCAN] / max(1, launches[sel.K_SCAN]) / 1e3
    achieved = mask_kernel_bytes / mask_avg_s / 1e9

    # the plain count query (no mask): kernel time and synchronous call latency
    prog = ctx.program(dt, tree)
    for _ in range(3):
        ctx.count(dt, prog)
    ctx.read_timing(reset=True)
    lat = []
    for _ in range(args.latency_reps):
        t1 = time.perf_counter()
        c2 = ctx.count(dt, prog)
        lat.append((time.perf_counter() - t1) * 1e3)
    ms2, l2 = ctx.read_timing(reset=True)
    count_avg_s = ms2[sel.K_COUNT] / max(1, l2[sel.K_COUNT]) / 1e3
    count_bytes = n * bpr
    assert c2 == cnt

    out = {
        "metric": "rows/s and HBM GB/s (% of peak) for exact filtered COUNT; p50/p99 estimate latency",
        "value": n * args.steps / elapsed,
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (seeded generator; TPC-H/SSB-like columns)",
        "config": {
            "workload": "fact table 300M rows x 8 columns (int32 date, int8 qty, int8 disc, "
                        "int64 log-normal price 5% NULL, 3 Zipf dictionary columns 7/25/4500, "
                        "int32 key); 6-leaf AND/OR predicate with a 10-code IN-list and a "
                        "4500-bit LIKE code bitmap; COUNT + limit check + ascending row ids",
            "rows": n,
            "selected_rows": cnt,
            "max_rows": max_rows,
            "bytes_per_row_read": bpr,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_scan<M_MASK> (evaluate + count + result mask)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_kernel_ms": mask_avg_s * 1e3,
            "algorithmic_bytes_per_launch": mask_kernel_bytes,
        },
        "count_query": {
            "kernel": "k_scan<M_COUNT>",
            "avg_kernel_ms": count_avg_s * 1e3,
            "rows_per_s": n / count_avg_s,
            "GBps": count_bytes / count_avg_s / 1e9,
            "frac_of_peak": count_bytes / count_avg_s / 1e9 / HBM_PEAK_GBS,
            "latency_ms_p50": percentile(lat, 50),
            "latency_ms_p99": percentile(lat, 99),
            "latency_reps": len(lat),
        },
        "step_kernels_ms": {"mask": mask_avg_s * 1e3, "tile_scan": scan_avg_s * 1e3,
                            "compact": compact_avg_s * 1e3},
    }

    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle over {n} rows on {threads} threads")
        c3, dt_cpu = cpu_baseline(table, tree, threads)
        assert c3 == cnt, (c3, cnt)
        out["cpu_baseline"] = {
            "value": n / dt_cpu,
            "unit": "rows/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"the full {n}-row table, COUNT only (the oracle's count), "
                      f"row ranges split over {threads} threads; {dt_cpu:.2f} s wall",
        }
    if args.copy_probe_mb:
        nb = args.copy_probe_mb << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        a.fill_(1)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"copy probe: {nb} bytes read and {nb} bytes written")
        del a, b
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
