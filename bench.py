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


def measured_traffic(kernels, profile="scan_fact300M_pushdown.md"):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated against a
    plain copy) of the named kernel, or summed over a list of kernels that
    one launch runs, from the committed rocprofv3 summary of this workload;
    None when the kernel source has changed since it was taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        src = open(os.path.join(root, "paper_1806_08384_amd", "csrc", "kernels.hip"), "rb").read()
        text = open(os.path.join(root, "profiles", profile)).read()
    except OSError:
        return None
    names = [kernels] if isinstance(kernels, str) else list(kernels)
    for line in text.splitlines():
        if line.startswith("traffic-json: "):
            rec = json.loads(line[len("traffic-json: "):])
            if rec.get("kernels_hip_sha256") != hashlib.sha256(src).hexdigest():
                return None
            per = rec.get("per_launch", {})
            if any(k not in per for k in names):
                return None
            return sum(per[k]["fetch_bytes"] + per[k]["write_bytes"] for k in names)
    return None


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def cpu_baseline(table, tree, threads):
    """The oracle as it stands, on this machine's host cores, over the same table
    (all rows, row ranges split over `threads` threads)."""
    import oracle
    orc = oracle.Oracle(table)
    t0 = time.perf_counter()
    c = orc.count(tree, threads=threads)
    dt = time.perf_counter() - t0
    return c, dt


def host_info():
    """The host the oracle runs on: logical CPUs, those this process may use,
    CPU model and memory."""
    info = {"logical_cpus": os.cpu_count(), "usable_cpus": host_threads()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["mem_total_gib"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def cpu_workloads(table, tree, threads, log):
    """The oracle on more of the workloads, each bounded to seconds: one
    thread on the first 20M rows of the fact table; the 1M-row three-column
    table; the 64 batching programs over their four tables (the fact table
    is the 300M one), all threads."""
    import numpy as np

    import datagen
    import oracle
    out = {}
    k = min(20_000_000, table.nrows) // 32 * 32
    sub = datagen.Table(f"fact[0:{k}]", k)
    for c in table.columns:
        v = None if c.valid is None else c.valid[: k // 32]
        sub.columns.append(datagen.Column(c.name, c.type, c.data[:k], v, c.dict_card))
    t0 = time.perf_counter()
    oracle.Oracle(sub).count(tree, threads=1)
    dt = time.perf_counter() - t0
    out["fact_one_thread"] = {"rows": sub.nrows, "threads": 1, "rows_per_s": sub.nrows / dt,
                              "wall_s": dt}
    u = datagen.cfg1(1_000_000)
    orc = oracle.Oracle(u)
    for th in (1, threads):
        t0 = time.perf_counter()
        for _ in range(20):
            orc.count(datagen.cfg1_predicate(), threads=th)
        dt = (time.perf_counter() - t0) / 20
        out[f"uniform3_1M_{th}_threads"] = {"rows": u.nrows, "threads": th,
                                            "rows_per_s": u.nrows / dt, "wall_s": dt}
    log("cpu baseline: the 64 batching programs")
    small = datagen.cfg3_tables(rows=datagen.CFG3_ROWS[:3], threads=threads)
    tabs = small + [table]
    orcs = [oracle.Oracle(t) for t in tabs]
    progs = datagen.cfg3_programs()
    t0 = time.perf_counter()
    for ti, tr in progs:
        orcs[ti].count(tr, threads=threads)
    dt = time.perf_counter() - t0
    prow = sum(tabs[ti].nrows for ti, _ in progs)
    out["batch_64_programs"] = {"program_rows": prow, "threads": threads,
                                "program_rows_per_s": prow / dt, "wall_s": dt}
    del small, tabs, orcs
    return out


def _timed(fn, reps):
    """Median wall time of fn() over reps runs, in ms (fn synchronises)."""
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = fn()
        ts.append((time.perf_counter() - t0) * 1e3)
    ts.sort()
    return ts[len(ts) // 2], r


def bench_batch(ctx, fact_dt, threads, log):
    """64 candidate predicates (2-8 leaves, selectivity 1e-5..0.9) over four
    tables of 10k / 2M / 60M / 300M rows: one persistent launch (eager and
    graph-replayed) against 64 plain count launches.  The 300M-row table is
    the resident fact table (same schema)."""
    import torch

    import datagen
    from paper_1806_08384_amd import sel
    log("batch: generating the 10k / 2M / 60M-row tables")
    small = datagen.cfg3_tables(rows=datagen.CFG3_ROWS[:3], threads=threads)
    dts = [sel.device_table(ctx, t) for t in small] + [fact_dt]
    progs = datagen.cfg3_programs()
    pairs = [(dts[t], ctx.program(dts[t], tree)) for t, tree in progs]
    reps = 5
    for _ in range(2):
        want = [ctx.count(t, p) for t, p in pairs]

    def plain_sync():
        return [ctx.count(t, p) for t, p in pairs]

    d_out = torch.zeros(len(pairs), dtype=torch.int64, device="cuda")

    def plain_async():
        for i, (t, p) in enumerate(pairs):
            ctx.count_async(t, p, d_out.data_ptr() + 8 * i)
        torch.cuda.synchronize()
        return d_out.cpu().tolist()

    def eager():
        return ctx.count_batch(pairs)

    b = ctx.batch(pairs)
    t_sync, r1 = _timed(plain_sync, reps)
    t_async, r2 = _timed(plain_async, reps)
    t_eager, r3 = _timed(eager, reps)
    ctx.read_timing(reset=True)
    t_graph, r4 = _timed(b.run, reps)
    bms, bl = ctx.read_timing(reset=True)
    graph_kernel_ms = bms[sel.K_BATCH] / max(1, bl[sel.K_BATCH])
    assert r1 == want and r2 == want and r3 == want and r4 == want, "batch counts differ"
    # algorithmic bytes of one launch: each table's rows times the union of
    # the columns its programs read (values, plus 1/8 B for the validity
    # bits of a nullable column)
    all_tables = list(small) + [None]
    union_bpr = []
    for ti in range(4):
        cols_used = set()
        for t, tree in progs:
            if t == ti:
                cols_used |= datagen.tree_columns(tree)
        if ti < 3:
            cols = all_tables[ti].columns
        else:
            cols = datagen.lineorder_like("schema", 1, 0).columns
        union_bpr.append(sum(datagen.WIDTH[cols[c].type] + (0.125 if cols[c].valid is not None else 0.0)
                             for c in cols_used))
    rows = [small[0].nrows, small[1].nrows, small[2].nrows, fact_dt.nrows]
    batch_bytes = sum(r * u for r, u in zip(rows, union_bpr))
    # bytes: plain reads each program's columns; the batch reads each table's
    # union of referenced columns once from HBM
    plain_bytes = sum(t.nrows * p.bytes_per_row for t, p in pairs)
    best_plain = min(t_sync, t_async)
    res = {
        "programs": len(pairs),
        "tables_rows": [int(datagen.CFG3_ROWS[0]), int(datagen.CFG3_ROWS[1]),
                        int(datagen.CFG3_ROWS[2]), int(fact_dt.nrows)],
        "plain_sync_ms": t_sync,
        "plain_async_ms": t_async,
        "batch_eager_ms": t_eager,
        "batch_graph_ms": t_graph,
        "speedup_vs_best_plain": best_plain / t_graph,
        "plain_bytes": plain_bytes,
        "counts_equal": True,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_luts + k_lbatch (and k_batch for programs outside conjunctive form), "
                      "graph replay",
            "algorithmic_bytes_per_launch": batch_bytes,
            "union_bytes_per_row": union_bpr,
            "avg_graph_ms": graph_kernel_ms,
            "achieved": batch_bytes / graph_kernel_ms / 1e6,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": batch_bytes / graph_kernel_ms / 1e6 / HBM_PEAK_GBS,
            # the graph's lookup-table launches (one per accumulator width)
            # and table builds, from the committed profile of this batch
            "traffic": measured_traffic(["k_lbatch<2, 8>", "k_lbatch<4, 4>", "k_luts"],
                                        "batch_64programs_4tables.md"),
        },
    }
    b.destroy()
    for t, p in pairs:
        p.destroy()
    return res, dts[:3]


def bench_star(ctx, fact_rows, threads, log, cpu=False):
    """Star push-down: dimension predicates become key bitmaps (2556 / 30k /
    200k / 3.2M-row dimensions), then the exact fact count by a conjunctive
    bitmap semi-join probe over a 480M-row fact table (4 int32 foreign keys)."""
    import torch

    import datagen
    from paper_1806_08384_amd import sel
    log(f"star: generating dimensions and a {fact_rows}-row fact table")
    dims = datagen.star_dims()
    preds = datagen.star_dim_predicates()
    fact = datagen.star_fact(fact_rows, threads=threads)
    ddims = [sel.device_table(ctx, d) for d in dims]
    dfact = sel.device_table(ctx, fact)
    cpu_star = None
    if cpu:
        import oracle
        log("star: the oracle's key bitmaps and star count")
        obms = [oracle.Oracle(d).keybitmap(p, 0, 0, d.nrows)[2] for d, p in zip(dims, preds)]
        t0 = time.perf_counter()
        oc = oracle.Oracle(fact).star_count([0, 1, 2, 3], obms, [d.nrows for d in dims],
                                            threads=threads)
        dt = time.perf_counter() - t0
        cpu_star = {"rows": fact_rows, "threads": threads, "rows_per_s": fact_rows / dt,
                    "wall_s": dt, "star_count": oc}
    del fact
    bitmaps, nbits, dim_ms, dim_counts = [], [], [], []
    for d, p in zip(ddims, preds):
        prog = ctx.program(d, p)
        bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
        ms, (st, c) = _timed(lambda: ctx.pushdown_keybitmap(d, 0, 0, prog, bm, d.nrows), 5)
        assert st == sel.SEL_OK
        bitmaps.append(bm)
        nbits.append(d.nrows)
        dim_ms.append(ms)
        dim_counts.append(c)
    fk = [0, 1, 2, 3]
    for _ in range(3):
        c = ctx.star_count(dfact, fk, bitmaps, nbits)
    ctx.read_timing(reset=True)
    reps = 10
    for _ in range(reps):
        c2 = ctx.star_count(dfact, fk, bitmaps, nbits)
    ms, l = ctx.read_timing(reset=True)
    assert c2 == c
    kms = ms[sel.K_STAR] / max(1, l[sel.K_STAR])
    bytes_ = fact_rows * 16
    res = {
        "fact_rows": fact_rows,
        "dim_rows": [d.nrows for d in ddims],
        "keybitmap_call_ms": dim_ms,
        "star_count": c,
        "star_kernel_ms": kms,
        "star_rows_per_s": fact_rows / (kms / 1e3),
        "star_GBps": bytes_ / (kms / 1e3) / 1e9,
        "star_frac_of_peak": bytes_ / (kms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "star_algorithmic_bytes": bytes_,
        # HBM bytes of one star launch from the committed profile (null if
        # the kernels changed since)
        "star_traffic": measured_traffic("star", "star_fact480M_probe.md"),
    }
    # the join order the exact dimension counts give (Ch.1 sec.1.1 formula)
    order, cost, inter = sel.star_plan(fact_rows, nbits, dim_counts)
    res["join_plan"] = {"dim_selected_rows": dim_counts, "order": order,
                        "intermediate_rows": inter, "formula_final_rows": inter[-1],
                        "exact_star_count": c, "intermediate_sum": cost}
    if cpu_star is not None:
        assert cpu_star["star_count"] == c, (cpu_star["star_count"], c)
        res["cpu_oracle"] = cpu_star
    return res, (dfact, ddims, dims)


def bench_achievable(log, gib=4, reps=10):
    """What plain streaming reaches on this GPU: a read-only reduction and a
    copy of a 4 GiB buffer (torch's kernels), timed with events on torch's
    stream; the lines against which the scan and the gather are read."""
    import torch
    n = (gib << 30) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)

    def rate(fn, nbytes):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        return {"ms": ms, "GBps": nbytes / ms / 1e6, "frac_of_peak": nbytes / ms / 1e6 / HBM_PEAK_GBS}

    res = {"bytes": 4 * n,
           "read_only_sum": rate(lambda: torch.sum(x), 4 * n),
           "copy": rate(lambda: y.copy_(x), 8 * n)}
    log(f"achievable: read {res['read_only_sum']['GBps']:.0f} GB/s, copy {res['copy']['GBps']:.0f} GB/s")
    del x, y
    torch.cuda.empty_cache()
    return res


def bench_gather(ctx, dt, table_cols, log, reps=5):
    """Projected columns of a materialised selection, gathered at its row
    ids on the 300M-row fact table: the 6-leaf predicate's ids (date, qty,
    price with NULLs, s25) and a date range selecting 90 % of the rows
    (date, price).  Algorithmic bytes per id: the id, each value read and
    written, and a nullable column's validity bit read and written."""
    import torch

    import datagen
    from paper_1806_08384_amd import sel
    width = {"i8": 1, "i16": 2, "i32": 4, "i64": 8}
    res = {}
    cases = [("P2 selection", datagen.cfg2_predicate(), [0, 1, 3, 5]),
             ("date range, 90% of rows", ("between", 0, 0, 2300), [0, 3])]
    for name, tree, cols in cases:
        prog = ctx.program(dt, tree)
        cnt = ctx.count(dt, prog)
        ids = torch.empty(max(1, cnt), dtype=torch.int32, device="cuda")
        st, c2 = ctx.pushdown_rowids(dt, prog, sel.UINT64_MAX, ids)
        assert st == sel.SEL_OK and c2 == cnt
        outs = [torch.empty(max(1, cnt), dtype=getattr(torch, {"i8": "int8", "i32": "int32",
                                                               "i64": "int64"}[table_cols[c][0]]),
                            device="cuda") for c in cols]
        vouts = [torch.empty(max(1, (cnt + 31) // 32), dtype=torch.int32, device="cuda")
                 if table_cols[c][1] else None for c in cols]
        ctx.gather(dt, ids, cnt, cols, outs, vouts)
        ctx.read_timing(reset=True)
        for _ in range(reps):
            ctx.gather(dt, ids, cnt, cols, outs, vouts)
        ms, l = ctx.read_timing(reset=True)
        kms = ms[sel.K_GATHER] / max(1, l[sel.K_GATHER])
        per_id = 4 + sum(2 * width[table_cols[c][0]] + (0.25 if table_cols[c][1] else 0) for c in cols)
        gbs = cnt * per_id / kms / 1e6
        res[name] = {"ids": cnt, "columns": [table_cols[c][2] for c in cols],
                     "bytes_per_id": per_id, "gather_kernel_ms": kms, "GBps": gbs,
                     "frac_of_peak": gbs / HBM_PEAK_GBS}
        log(f"gather, {name}: {cnt} ids x {len(cols)} columns, {kms:.3f} ms, {gbs:.0f} GB/s")
        del ids, outs, vouts
    torch.cuda.empty_cache()
    return res


def bench_estimate_error(ctx, small, fact_dt, log):
    """What exact counting replaces (Ch.1 sec.1.1): for the 6-leaf fact
    predicate and for the 64 batching programs, the product of the
    conjuncts' selectivities (the independence estimate) against the exact
    count, from each program's conjunct counts (one batched launch each)."""
    import datagen
    dts = list(small) + [fact_dt]
    prog = ctx.program(fact_dt, datagen.cfg2_predicate())
    c, fc = ctx.factor_counts(fact_dt, prog)
    est = ctx.independence_estimate(fact_dt.nrows, fc)
    qs = []
    t0 = time.perf_counter()
    for ti, tree in datagen.cfg3_programs():
        p = ctx.program(dts[ti], tree)
        cc, ff = ctx.factor_counts(dts[ti], p)
        e = ctx.independence_estimate(dts[ti].nrows, ff)
        qs.append(max(max(e, 1.0) / max(cc, 1.0), max(cc, 1.0) / max(e, 1.0)))
    dt = time.perf_counter() - t0
    qs.sort()
    q = lambda f: qs[min(len(qs) - 1, int(round(f * (len(qs) - 1))))]
    log(f"estimate error: fact predicate exact {c}, independence {est:.0f}; "
        f"64 programs q-error median {q(0.5):.2f}, max {qs[-1]:.1f}")
    return {
        "fact_predicate": {"rows": fact_dt.nrows, "exact": c, "conjunct_counts": fc,
                           "independence_estimate": est,
                           "q_error": max(max(est, 1.0) / max(c, 1.0), max(c, 1.0) / max(est, 1.0))},
        "batch_64_programs": {"q_error_median": q(0.5), "q_error_p90": q(0.9),
                              "q_error_max": qs[-1], "calls_s": dt},
    }


def bench_autotune(ctx, dt, tree, small, log):
    """The tuner (per kernel, program class and table size: workgroup size
    and count, then cached or nontemporal loads, tiles per wave step and the
    LDS staging limit for the scans, rows per lane for the lookup-table
    batch kernel) on the step's scans and on the 64-program batch, beside
    the defaults measured above; each knob's pick is reported with whether
    the library default already equals it.  It runs last: the tuned
    configurations stay on the context."""
    import datagen
    from paper_1806_08384_amd import sel
    prog = ctx.program(dt, tree)
    out = {}
    # the library defaults for a scan: 256-thread workgroups, 12 resident
    # waves per CU, nontemporal loads, one tile per step, all staging
    default_scan = {"block": 256, "grid": 3 * ctx.num_cus, "cached": 0, "tiles_per_step": 1, "stage_words": 0}
    for name, mask in (("k_scan<M_MASK>", True), ("k_scan<M_COUNT>", False)):
        cfg, ms = ctx.autotune(dt, prog, with_mask=mask, reps=5)
        pick = {k: getattr(cfg, k) for k in ("block", "grid", "cached", "tiles_per_step", "stage_words")}
        out[name] = {**pick, "tuned_kernel_ms": ms,
                     "default_is_pick": {k: default_scan[k] == v for k, v in pick.items()}}
        log(f"autotune {name}: {pick}, {ms:.3f} ms")
    if small is not None:
        dts = list(small) + [dt]
        pairs = [(dts[t], ctx.program(dts[t], tr)) for t, tr in datagen.cfg3_programs()]
        cfg, ms = ctx.autotune_batch(pairs, reps=3)
        pick = {"block": cfg.block, "grid": cfg.grid, "rows_per_lane": cfg.rows_per_lane or 8}
        out["batch (64 programs, eager call)"] = {**pick, "tuned_call_ms": ms,
                                                  "default_is_pick": {"rows_per_lane": pick["rows_per_lane"] == 8}}
        log(f"autotune batch: {pick}, {ms:.3f} ms")
    return out


def bench_select_pushdown(ctx, small, fact_dt, star, log, reps=10):
    """Algorithm 1's whole decision (size queue, probe skipped, exact count,
    limit, ids of each pushed relation) on two queries: the star schema
    (480M-row fact table probed, four dimensions evaluated) and the four
    fact-schema tables (300M probed; 60M, 2M and 10k rows evaluated), at
    PUSH_DOWN_MAX_SELECTIVITY 0.05 and PUSH_DOWN_MIN_TABLE_SIZE 1000."""
    import torch

    import datagen
    from paper_1806_08384_amd import sel
    dfact, ddims, _ = star
    queries = {
        "star_480M_fact_4_dims": [(dfact, None)] + list(zip(ddims, datagen.star_dim_predicates())),
        "fact_tables_300M_60M_2M_10k": [(fact_dt, datagen.cfg2_predicate())] + [
            (t, datagen.cfg2_predicate(0, 1000)) for t in small],
    }
    out = {}
    for name, rels in queries.items():
        args = []
        for t, tree in rels:
            buf = torch.empty(max(1, sel.max_rows(t.nrows, 0.05)), dtype=torch.int32, device="cuda")
            args.append((t, ctx.program(t, tree) if tree is not None else None, buf))
        ctx.select_pushdown(args)
        ms, res = _timed(lambda: ctx.select_pushdown(args), reps)
        out[name] = {
            "relations_rows": [t.nrows for t, _ in rels],
            "decisions": [r["decision"] for r in res],
            "counts": [r["count"] for r in res],
            "max_rows": [r["max_rows"] for r in res],
            "call_ms_median": ms,
        }
        log(f"algorithm 1, {name}: {ms:.3f} ms, {[r['decision'] for r in res]}")
        del args
    torch.cuda.empty_cache()
    return out


def bench_serve(ctx, small, fact_dt, star, threads, log, seconds, server_cfg=None):
    """Poisson stream (2000 requests/s) of estimate requests, 1-12 programs
    each over the resident tables (1M uniform, 2M, 60M, the 300M fact table
    and the 480M star fact table), 10 % with a push-down with row ids, served
    with continuous batching after a 1 s warm-up; against serial plain calls
    (FIFO) on the first second of the same arrival trace."""
    import threading

    import torch

    import datagen
    from paper_1806_08384_amd import sel
    dfact, ddims, dims = star
    log("serve: building the 1M table and program pools")
    t1m = sel.device_table(ctx, datagen.cfg1(1_000_000, seed=51, threads=threads))
    tables = [t1m, small[1], small[2], fact_dt, dfact]
    pools = [[ctx.program(t1m, t) for t in datagen.uniform3_programs(52, 32)]]
    for k, tb in ((1, small[1]), (2, small[2]), (3, fact_dt)):
        trees = [tree for _, tree in datagen.cfg3_programs(seed=60 + k, per_table=32, ntables=1)]
        pools.append([ctx.program(tb, t) for t in trees])
    star_pool, keep = [], []
    for combo in datagen.star_dim_programs(53, 16, dims):
        bms = []
        for d, p in zip(ddims, combo):
            bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
            st, _ = ctx.pushdown_keybitmap(d, 0, 0, ctx.program(d, p), bm, d.nrows)
            assert st == sel.SEL_OK
            bms.append(bm)
        keep.append(bms)
        star_pool.append(ctx.star_program(dfact, [0, 1, 2, 3], bms, [d.nrows for d in ddims]))
    pools.append(star_pool)
    alone = [[ctx.count(tables[k], p) for p in pool] for k, pool in enumerate(pools)]
    warm = 1.0
    trace = datagen.serving_trace(seed=52, rate=2000.0, duration=warm + seconds,
                                  pool_sizes=tuple(len(p) for p in pools))
    n_warm = sum(1 for t, _, _ in trace if t < warm)
    pd_bufs = {}
    for tb in range(4):
        mx = sel.max_rows(tables[tb].nrows, 0.05)
        pd_bufs[tb] = (mx, [torch.empty(max(1, mx), dtype=torch.int32, device="cuda")
                            for _ in range(4)])
    srv = ctx.server(**({"hbm_budget_bytes": 4 << 30} | dict(server_cfg or {})))
    tickets = [None] * len(trace)
    err = []

    def client():
        t0 = time.perf_counter()
        try:
            for i, (t, items, pd) in enumerate(trace):
                while True:
                    dt_ = t - (time.perf_counter() - t0)
                    if dt_ <= 0:
                        break
                    time.sleep(dt_ if dt_ > 0.002 else 0)
                pairs = [(tables[tb], pools[tb][pi]) for tb, pi in items]
                pdarg = None
                if pd is not None:
                    tb, pi = pd
                    mx, bufs = pd_bufs[tb]
                    pdarg = (tables[tb], pools[tb][pi], mx, bufs[i % len(bufs)])
                tickets[i] = srv.submit(pairs, pdarg)
                if i + 1 == n_warm:
                    srv.stats(reset=True)
        except Exception as e:
            err.append(e)

    log(f"serve: {len(trace)} requests over {warm + seconds:.0f} s")
    th = threading.Thread(target=client)
    th.start()
    lat, mismatches, by_big, by_pd = [], 0, {}, {}
    for i in range(len(trace)):
        while tickets[i] is None and not err:
            time.sleep(0.0002)
        if err:
            break
        counts, st, pdc, ms = srv.wait(tickets[i])
        if counts != [alone[tb][pi] for tb, pi in trace[i][1]]:
            mismatches += 1
        if i >= n_warm:
            lat.append(ms)
            big = max([tables[tb].nrows for tb, _ in trace[i][1]] +
                      ([tables[trace[i][2][0]].nrows] if trace[i][2] else []))
            by_big.setdefault(big, []).append(ms)
            by_pd.setdefault("with_pushdown" if trace[i][2] else "counts_only", []).append(ms)
    th.join()
    if err:
        raise err[0]
    stats = srv.stats()
    srv.destroy()
    assert mismatches == 0, f"{mismatches} served results differ from the same requests alone"

    # serial plain launches on the first second of the same trace
    n_serial = min(len(trace), 2000)
    log(f"serve: serial baseline over {n_serial} requests")
    service = []
    for i in range(n_serial):
        t, items, pd = trace[i]
        t0 = time.perf_counter()
        for tb, pi in items:
            ctx.count(tables[tb], pools[tb][pi])
        if pd is not None:
            tb, pi = pd
            mx, bufs = pd_bufs[tb]
            ctx.pushdown_rowids(tables[tb], pools[tb][pi], mx, bufs[0])
        service.append(time.perf_counter() - t0)
    finish, serial_lat = 0.0, []
    for i in range(n_serial):
        start = max(trace[i][0], finish)
        finish = start + service[i]
        serial_lat.append((finish - trace[i][0]) * 1e3)
    serial_lat.sort()
    res = {
        "rate_per_s": 2000.0,
        "requests": len(trace) - n_warm,
        "programs_per_request_mean": sum(len(x[1]) for x in trace) / len(trace),
        "pushdown_fraction": sum(1 for x in trace if x[2]) / len(trace),
        "throughput_req_per_s": stats["completed"] / stats["elapsed_s"] if stats["elapsed_s"] else None,
        "p50_ms": stats["p50_ms"],
        "p99_ms": stats["p99_ms"],
        "mean_ms": stats["mean_ms"],
        "max_ms": stats["max_ms"],
        "rounds": stats["rounds"],
        "programs_per_round": stats["round_programs"] / max(1, stats["rounds"]),
        "distinct_programs_per_round": stats["round_groups"] / max(1, stats["rounds"]),
        "round_gpu_ms_mean": stats["round_gpu_ms"] / max(1, stats["rounds"]),
        "round_host_ms_mean": stats["round_host_ms"] / max(1, stats["rounds"]),
        "gpu_busy_fraction": (stats["round_gpu_ms"] / (stats["elapsed_s"] * 1e3)
                              if stats["elapsed_s"] else None),
        # per round: the chunk rows of each table times the columns its
        # programs read, over the round's device time
        "round_bytes_mean": stats["round_bytes"] / max(1, stats["rounds"]),
        "round_GBps": (stats["round_bytes"] / stats["round_gpu_ms"] / 1e6
                       if stats["round_gpu_ms"] else None),
        "round_frac_of_peak": (stats["round_bytes"] / stats["round_gpu_ms"] / 1e6 / HBM_PEAK_GBS
                               if stats["round_gpu_ms"] else None),
        "by_largest_table_rows": {
            str(k): {"requests": len(v), "p50_ms": percentile(sorted(v), 50),
                     "p99_ms": percentile(sorted(v), 99)}
            for k, v in sorted(by_big.items())},
        "by_pushdown": {
            k: {"requests": len(v), "p50_ms": percentile(sorted(v), 50),
                "p99_ms": percentile(sorted(v), 99)}
            for k, v in sorted(by_pd.items())},
        "shared_rounds": stats["shared_rounds"],
        "max_admitted": stats["max_admitted"],
        "results_equal_alone": True,
        "serial_plain": {
            "requests": n_serial,
            "throughput_req_per_s": n_serial / sum(service),
            "p50_ms": percentile(serial_lat, 50),
            "p99_ms": percentile(serial_lat, 99),
        },
    }
    return res


def bench_sweeps(ctx, dt, n, threads, log, in_lists, reps=3):
    """Count-kernel rate against selectivity and against the number of leaves
    on the 300M-row fact table (the analogues of the thesis' overhead versus
    selectivity and versus attribute count experiments), with the push-down
    step (count + mask, limit, scan, ascending ids) at each selectivity; and
    the three-column uniform table at 300M rows, a pure bandwidth probe.
    Each count is timed in the configuration the tuner picks for its program
    class (reported per row as `launch`); the push-down step keeps the
    defaults."""
    import torch

    import datagen
    from paper_1806_08384_amd import sel

    tuned = {}

    def count_ms(table, prog):
        # the count scan in the configuration the tuner picks for this
        # program class and table size (a deployment tunes each class once)
        cfg, _ = ctx.autotune(table, prog, with_mask=False, reps=3)
        tuned[id(prog)] = {k: getattr(cfg, k) for k in ("block", "grid", "cached", "tiles_per_step", "stage_words")}
        ctx.count(table, prog)
        ctx.read_timing(reset=True)
        for _ in range(reps):
            c = ctx.count(table, prog)
        ms, l = ctx.read_timing(reset=True)
        return c, ms[sel.K_COUNT] / max(1, l[sel.K_COUNT])

    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    sel_rows = []
    cases = [("P2, date window %d days" % w, datagen.cfg2_predicate(365, 365 + w - 1))
             for w in (1, 10, 100, 365)]
    cases.append(("P2, every date", datagen.cfg2_predicate(0, 2556)))
    cases += [("date range, %d%% of days" % int(100 * f), ("between", 0, 0, int(round(f * 2557)) - 1))
              for f in (0.1, 0.3, 0.6, 0.9)]
    for name, tree in cases:
        prog = ctx.program(dt, tree)
        c, kms = count_ms(dt, prog)
        bpr = prog.bytes_per_row
        st, cnt = ctx.pushdown_rowids(dt, prog, sel.UINT64_MAX, ids)
        assert st == sel.SEL_OK and cnt == c, (st, cnt, c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.pushdown_rowids(dt, prog, sel.UINT64_MAX, ids)
        torch.cuda.synchronize()
        pd_ms = (time.perf_counter() - t0) / reps * 1e3
        gbs = n * bpr / kms / 1e6
        sel_rows.append({"program": name, "selected_rows": c, "selectivity": c / n, "launch": tuned[id(prog)],
                         "count_kernel_ms": kms, "count_GBps": gbs,
                         "count_frac_of_peak": gbs / HBM_PEAK_GBS,
                         "pushdown_step_ms": pd_ms, "ids_bytes": 4 * c})
        log(f"sweep: {name}: selectivity {c / n:.2e}, count {kms:.3f} ms, push-down {pd_ms:.3f} ms")
    del ids
    torch.cuda.empty_cache()

    leaves = [("between", 0, 0, 1999), ("cmp", 1, "<", 45), ("between", 2, 0, 9),
              ("cmp", 3, ">=", 2000), ("in", 5, tuple(range(0, 24))),
              ("codeset", 6, 4500, datagen.cfg2_like_bitmap() | 0xAAAAAAAA),
              ("in", 4, (0, 1, 2, 3, 4, 5)), ("cmp", 0, ">=", 10)]
    leaf_rows = []
    for k in range(1, len(leaves) + 1):
        tree = leaves[0] if k == 1 else ("and", *leaves[:k])
        prog = ctx.program(dt, tree)
        c, kms = count_ms(dt, prog)
        bpr = prog.bytes_per_row
        gbs = n * bpr / kms / 1e6
        leaf_rows.append({"leaves": k, "bytes_per_row": bpr, "selected_rows": c, "launch": tuned[id(prog)],
                          "count_kernel_ms": kms, "rows_per_s": n / kms * 1e3,
                          "count_GBps": gbs, "count_frac_of_peak": gbs / HBM_PEAK_GBS})
        log(f"sweep: {k} leaves, {bpr} B/row: count {kms:.3f} ms, {gbs:.0f} GB/s")

    # sparse IN lists of 10, 100 and 1000 values on the int64 price column
    # (5 % NULLs; half the values occur): sorted lists searched in the
    # scan's LDS copy
    in_rows = []
    for k, values in sorted(in_lists.items()):
        tree = ("in", 3, values)
        prog = ctx.program(dt, tree)
        c, kms = count_ms(dt, prog)
        bpr = prog.bytes_per_row
        gbs = n * bpr / kms / 1e6
        in_rows.append({"list_values": k, "present_values": k // 2, "bytes_per_row": bpr, "selected_rows": c,
                        "launch": tuned[id(prog)],
                        "count_kernel_ms": kms, "count_GBps": gbs, "count_frac_of_peak": gbs / HBM_PEAK_GBS})
        log(f"sweep: int64 IN list of {k} values: {c} rows, {kms:.3f} ms, {gbs:.0f} GB/s")
        prog.destroy()

    log("sweep: three uniform int32 columns at 300M rows")
    u = datagen.cfg1(n=300_000_000, threads=threads)
    du = sel.device_table(ctx, u)
    del u
    prog = ctx.program(du, datagen.cfg1_predicate())
    c, kms = count_ms(du, prog)
    gbs = du.nrows * prog.bytes_per_row / kms / 1e6
    uni = {"rows": du.nrows, "bytes_per_row": prog.bytes_per_row, "selected_rows": c,
           "count_kernel_ms": kms, "count_GBps": gbs, "count_frac_of_peak": gbs / HBM_PEAK_GBS}
    del du, prog
    torch.cuda.empty_cache()
    return {"selectivity": sel_rows, "leaves": leaf_rows, "in_list_int64": in_rows, "uniform3_300M": uni}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rows", type=int, default=300_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-reps", type=int, default=50)
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-predicate batching measurement")
    ap.add_argument("--no-star", action="store_true",
                    help="skip the star-schema push-down measurement")
    ap.add_argument("--star-rows", type=int, default=480_000_000)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving (Poisson request stream) measurement")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--no-sweeps", action="store_true",
                    help="skip the selectivity / leaf-count sweeps and the bandwidth probe")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip everything beyond the step, the count query, the batch, the star "
                         "probe and serving (sweeps, gather, achievable rates, estimate error, "
                         "Algorithm 1), e.g. to profile those kernels alone")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB once (a plain "
                         "copy kernel of known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1",
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
    # the mask pass writes the result words that hold a TRUE row (lane L of
    # a 2048-row tile holds rows 256 j + 4 L + i), and 12 B per tile (count
    # and lane map); the words are counted from the ids the step returned
    idv = ids[:cnt].to(torch.int64) & 0xFFFFFFFF
    mask_words = int(torch.unique((idv // 2048) * 64 + (idv % 256) // 4).numel())
    del idv
    mask_kernel_bytes = n * bpr + 4 * mask_words + ntiles * 12
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
            "traffic": measured_traffic("k_scan<1, true>"),
            "avg_kernel_ms": mask_avg_s * 1e3,
            "algorithmic_bytes_per_launch": mask_kernel_bytes,
            "mask_words_written": mask_words,
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
            "host": host_info(),
            "per_workload": cpu_workloads(table, tree, threads, log),
        }
    table_cols = [(c.type, c.valid is not None, c.name) for c in table.columns]
    # sparse IN lists for the sweep, drawn from the price column
    in_lists = {k: datagen.sparse_in_values(table.col("price").data, k) for k in (10, 100, 1000)}
    del table
    if not args.no_extras:
        out["gather"] = bench_gather(ctx, dt, table_cols, log)
        out["achievable"] = bench_achievable(log)
    if not args.no_sweeps and not args.no_extras:
        out["sweeps"] = bench_sweeps(ctx, dt, n, threads, log, in_lists)
    small = star = None
    if not args.no_batch:
        out["batch"], small = bench_batch(ctx, dt, threads, log)
    if not args.no_star:
        out["star"], star = bench_star(ctx, args.star_rows, threads, log,
                                       cpu="cpu_baseline" in out)
        if "cpu_oracle" in out["star"]:
            out["cpu_baseline"]["per_workload"]["star_480M"] = out["star"].pop("cpu_oracle")
    if small is not None and not args.no_extras:
        out["estimate_error"] = bench_estimate_error(ctx, small, dt, log)
    if small is not None and star is not None and not args.no_extras:
        out["select_pushdown"] = bench_select_pushdown(ctx, small, dt, star, log)
    if not args.no_serve and small is not None and star is not None:
        out["serving"] = bench_serve(ctx, small, dt, star, threads, log, args.serve_seconds)
    if not args.no_extras:
        out["autotune"] = bench_autotune(ctx, dt, tree, small, log)
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
