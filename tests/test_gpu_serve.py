"""GPU: the serving loop (continuous batching with cooperative scans).
Every request's results in a mixed, overlapping stream equal the oracle's
(counts exact, row ids bit-identical) and so its results alone, and
admission by device footprint holds requests back or rejects them without
failing."""
import threading
import time

import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_common import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sel():
    if not torch.cuda.is_available():
        pytest.fail("gpu test run without a GPU")
    from paper_1806_08384_amd import sel as s
    return s


@pytest.fixture(scope="module")
def ctx(sel):
    c = sel.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.fixture(scope="module")
def world(sel, ctx):
    """Five resident tables (a uniform int32 table, three fact-schema tables
    and a star fact table with four dimensions) and a program pool each.
    `want` holds the oracle's count of every pool program; `alone` the
    library's plain count of it, which must equal it."""
    say("serve: building tables and pools")
    host = [datagen.cfg1(200_000, seed=7),
            datagen.lineorder_like("t1", 300_000, 32),
            datagen.lineorder_like("t2", 1_000_003, 33),
            datagen.lineorder_like("t3", 3_000_000, 2)]
    dim_rows = (2556, 3000, 20_000, 32_000)
    dims = datagen.star_dims(seed=42, sizes=dim_rows)
    fact = datagen.star_fact(2_000_000, dim_rows=dim_rows)
    dts = [sel.device_table(ctx, t) for t in host]
    dfact = sel.device_table(ctx, fact)
    ddims = [sel.device_table(ctx, d) for d in dims]
    trees = [datagen.uniform3_programs(11, 16)]
    for k in (1, 2, 3):
        trees.append([tree for _, tree in datagen.cfg3_programs(seed=100 + k, per_table=16,
                                                                ntables=1)])
    pools = [[ctx.program(dts[k], t) for t in trees[k]] for k in range(4)]
    orcs = [oracle.Oracle(t) for t in host]
    want = [[orcs[k].count(t, threads=8) for t in trees[k]] for k in range(4)]
    star_pool, star_want, keep = [], [], []
    ofact = oracle.Oracle(fact)
    for combo in datagen.star_dim_programs(9, 8, dims):
        bms, bms_cpu, nbits = [], [], []
        for d, hd, p in zip(ddims, dims, combo):
            bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
            st, _ = ctx.pushdown_keybitmap(d, 0, 0, ctx.program(d, p), bm, d.nrows)
            assert st == sel.SEL_OK
            ost, _, owords = oracle.Oracle(hd).keybitmap(p, 0, 0, hd.nrows)
            assert ost == 0
            bms.append(bm)
            bms_cpu.append(owords)
            nbits.append(d.nrows)
        keep.append(bms)
        star_pool.append(ctx.star_program(dfact, [0, 1, 2, 3], bms, nbits))
        star_want.append(ofact.star_count([0, 1, 2, 3], bms_cpu, nbits, threads=8))
    pools.append(star_pool)
    want.append(star_want)
    tables = dts + [dfact]
    alone = [[ctx.count(tables[k], p) for p in pool] for k, pool in enumerate(pools)]
    assert alone == want
    return dict(tables=tables, pools=pools, alone=alone, want=want, keep=keep, host=host,
                trees=trees, orcs=orcs)


def run_trace(sel, ctx, world, trace, srv, time_scale=1.0):
    """Submit the trace at its (scaled) arrival times from a client thread;
    return [(counts, pd_status, pd_count, latency, ids)] in trace order."""
    tables, pools = world["tables"], world["pools"]
    tickets = [None] * len(trace)
    outs = [None] * len(trace)
    err = []

    def client():
        t0 = time.perf_counter()
        try:
            for i, (t, items, pd) in enumerate(trace):
                while time.perf_counter() - t0 < t * time_scale:
                    time.sleep(0.0001)
                pairs = [(tables[tb], pools[tb][pi]) for tb, pi in items]
                pdarg = None
                if pd is not None:
                    tb, pi = pd
                    mx = sel.max_rows(tables[tb].nrows, 0.05)
                    out = torch.full((max(1, mx),), -1, dtype=torch.int32, device="cuda")
                    outs[i] = out
                    pdarg = (tables[tb], pools[tb][pi], mx, out)
                tickets[i] = srv.submit(pairs, pdarg)
        except Exception as e:  # surfaced by the main thread
            err.append(e)

    th = threading.Thread(target=client)
    th.start()
    results = []
    for i in range(len(trace)):
        while tickets[i] is None and not err:
            time.sleep(0.0001)
        if err:
            break
        counts, st, pdc, lat = srv.wait(tickets[i])
        results.append((counts, st, pdc, lat, outs[i]))
    th.join()
    if err:
        raise err[0]
    return results


def test_mix_equals_alone(sel, ctx, world):
    trace = datagen.serving_trace(seed=5, rate=4000.0, duration=0.1,
                                  pool_sizes=(16, 16, 16, 16, 8))
    say(f"serve: {len(trace)} requests")
    srv = ctx.server(chunk_rows=1 << 18, hbm_budget_bytes=1 << 30)
    res = run_trace(sel, ctx, world, trace, srv)
    stats = srv.stats()
    tables, want = world["tables"], world["want"]
    checked = 0
    for (t, items, pd), (counts, st, pdc, lat, out) in zip(trace, res):
        assert counts == [want[tb][pi] for tb, pi in items]
        if pd is not None:
            tb, pi = pd
            mx = sel.max_rows(tables[tb].nrows, 0.05)
            ost, ocnt, oids = world["orcs"][tb].pushdown(world["trees"][tb][pi], mx,
                                                         max(1, mx))
            assert (st, pdc) == ({0: sel.SEL_OK, 1: sel.SEL_OVER_LIMIT}[ost], ocnt)
            got = out.cpu().numpy().view(np.uint32)
            if ost == 0:
                np.testing.assert_array_equal(got[:ocnt], oids)
                got = got[ocnt:]
            assert np.all(got == 0xFFFFFFFF)   # nothing past the ids, nothing over the limit
            checked += 1
    say(f"serve: {checked} push-downs checked against the oracle")
    assert stats["completed"] == len(trace)
    # work of different requests overlapped: shared scans, several admitted
    assert stats["shared_rounds"] > 0 and stats["max_admitted"] > 1
    say(f"serve stats: {stats}")
    srv.destroy()


def test_single_request_alone(sel, ctx, world):
    tables, pools, alone = world["tables"], world["pools"], world["want"]
    srv = ctx.server()
    for tb in range(5):
        tk = srv.submit([(tables[tb], pools[tb][1])])
        counts, st, pdc, lat = srv.wait(tk)
        assert counts == [alone[tb][1]] and st == sel.SEL_OK and lat > 0
    # a push-down only request
    mx = sel.max_rows(tables[3].nrows, 0.5)
    out = torch.empty(mx, dtype=torch.int32, device="cuda")
    tk = srv.submit([], (tables[3], pools[3][0], mx, out))
    counts, st, pdc, lat = srv.wait(tk)
    assert counts == [] and pdc == alone[3][0]
    srv.destroy()


def test_admission_by_footprint(sel, ctx, world):
    """A tiny budget: a request larger than the budget is rejected; requests
    that fit alone but not together wait for each other; all finish."""
    tables, pools, alone = world["tables"], world["pools"], world["want"]
    srv = ctx.server(hbm_budget_bytes=12_000, chunk_rows=1 << 18)
    out = torch.empty(1000, dtype=torch.int32, device="cuda")
    with pytest.raises(sel.SelError) as ei:
        srv.submit([], (tables[3], pools[3][0], 1000, out))   # mask alone > budget
    assert ei.value.status == sel.SEL_E_BUSY
    rng = np.random.default_rng(1)
    reqs = []
    for _ in range(40):
        items = [(int(rng.integers(0, 5)), int(rng.integers(0, 8))) for _ in range(8)]
        reqs.append(items)
    tks = [srv.submit([(tables[tb], pools[tb][pi]) for tb, pi in it]) for it in reqs]
    for it, tk in zip(reqs, tks):
        counts, st, pdc, lat = srv.wait(tk)
        assert counts == [alone[tb][pi] for tb, pi in it]
    stats = srv.stats()
    assert stats["rejected"] == 1
    assert stats["max_admitted"] < 40          # the budget held requests back
    srv.destroy()


def test_chunk_sizes_agree(sel, ctx, world):
    """The same requests with one chunk per table and with many chunks
    (equal chunks per table, and chunks capped by a row count)."""
    tables, pools, alone = world["tables"], world["pools"], world["want"]
    trace = datagen.serving_trace(seed=8, rate=2000.0, duration=0.03,
                                  pool_sizes=(16, 16, 16, 16, 8), pushdown_rate=0.0)
    for cycle, chunk in ((1, 0), (8, 0), (3, 1 << 16), (1000, 2048)):
        srv = ctx.server(chunk_rows=chunk, rounds_per_cycle=cycle, rounds_in_flight=3)
        res = run_trace(sel, ctx, world, trace, srv, time_scale=0.0)
        for (t, items, pd), (counts, *_rest) in zip(trace, res):
            assert counts == [alone[tb][pi] for tb, pi in items], (cycle, chunk)
        srv.destroy()


def test_table_recreated_at_same_address(sel, ctx):
    """A table destroyed while the server lives and a larger one created in
    its place (the allocator usually hands back the same address): the
    server scans the new table's rows, not the old geometry."""
    small = datagen.lineorder_like("s", 100_003, 61)
    big = datagen.lineorder_like("b", 1_500_001, 62)
    tree = ("between", 0, 100, 1900)
    srv = ctx.server(rounds_per_cycle=3)
    addrs = []
    for host in (small, big, small):
        dt = sel.device_table(ctx, host)
        addrs.append(dt.h.value)
        prog = ctx.program(dt, tree)
        counts, st, pdc, lat = srv.wait(srv.submit([(dt, prog)]))
        assert counts == [oracle.Oracle(host).count(tree, threads=8)], host.name
        prog.destroy()
        dt.destroy()
    say(f"serve: table addresses {[hex(a) for a in addrs]}")
    srv.destroy()
