"""GPU: the push-down decision of Algorithm 1 (sel_select_pushdown through
the C ABI) against the oracle's step-by-step EvaluateAndPushDown: the same
decisions, queue order, exact counts, limits and ascending row ids; and the
conjunct counts behind the independence estimate (sel_factor_counts)."""
import numpy as np
import pytest

import datagen
import oracle
from tests import sqlite_ref
from tests.gpu_common import as_u32, ids_tensor, say

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


def run_both(sel, ctx, tables, trees, caps, min_size, ratio):
    dts = [sel.device_table(ctx, t) for t in tables]
    rels, bufs = [], []
    for dt, tree, cap in zip(dts, trees, caps):
        buf = ids_tensor(cap, torch) if cap > 0 else None
        bufs.append(buf)
        rels.append((dt, ctx.program(dt, tree) if tree is not None else None, buf))
    got = ctx.select_pushdown(rels, min_table_size=min_size, max_selectivity=ratio)
    want = oracle.select_pushdown([(t, tree, cap) for t, tree, cap in zip(tables, trees, caps)],
                                  min_table_size=min_size, max_selectivity=ratio)
    for i, (g, w) in enumerate(zip(got, want)):
        assert (g["decision"], g["order"], g["count"], g["max_rows"], g["status"]) == \
            (w["decision"], w["order"], w["count"], w["max_rows"], w["status"]), (i, g, w)
        if w["decision"] == "pushed":
            np.testing.assert_array_equal(as_u32(bufs[i])[:g["count"]], w["ids"])
    return got


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_spd_random_relations(sel, ctx, seed):
    """Random relations of ragged sizes (some equal, some at the threshold,
    some without a selection) with random predicates under NULLs, at a ratio
    that pushes some and reverts others; one buffer too small."""
    say(f"spd random seed={seed}")
    rng = np.random.default_rng(70_000 + seed)
    sizes = [int(x) for x in rng.choice([500, 1000, 1001, 4097, 20_000, 65_537, 150_001], 7)]
    sizes[int(rng.integers(0, 7))] = sizes[0]          # a tie
    tables = [datagen.random_table(rng, n, grid=bool(k % 2), null_rate=0.2)
              for k, n in enumerate(sizes)]
    trees = [None if rng.random() < 0.15 else
             sqlite_ref.clamp_literals(datagen.random_tree(rng, t, grid=bool(k % 2)))
             for k, t in enumerate(tables)]
    caps = [n for n in sizes]
    caps[int(rng.integers(0, 7))] = 3                  # pushed only if at most 3 rows
    ratio = float(rng.choice([0.05, 0.2, 0.5]))
    got = run_both(sel, ctx, tables, trees, caps, 1000, ratio)
    assert sum(1 for g in got if g["decision"] == "probe") == (1 if max(sizes) > 1000 else 0)


def test_spd_forced_limits(sel, ctx):
    """The limit on either side of each relation's count: maxSize = count - 1
    reverts, count and count + 1 push (ratios j / 8192 on 8192-row
    relations make maxSize exactly j)."""
    rng = np.random.default_rng(71_000)
    probe = datagen.random_table(rng, 20_000, grid=False, null_rate=0.1)
    t = datagen.random_table(rng, 8192, grid=False, null_rate=0.1)
    tree = ("and", ("cmp", 0, ">=", -5), ("cmp", 3, "<", 12))
    c = oracle.Oracle(t).count(tree)
    assert 0 < c < 8191
    for j, want in ((c - 1, "reverted"), (c, "pushed"), (c + 1, "pushed")):
        got = run_both(sel, ctx, [probe, t], [None, tree], [0, 8192], 1000, j / 8192)
        assert got[1]["decision"] == want and got[1]["max_rows"] == j


def test_spd_star_schema(sel, ctx):
    """A star query: a 10M-row fact table (the probe) and the four dimension
    tables (2556 / 30k / 200k / 3.2M rows) with their predicates at the 5 %
    limit: the largest dimension is pushed, the others revert."""
    say("spd star: generating")
    dims = datagen.star_dims()
    fact = datagen.star_fact(10_000_000, threads=16)
    tables = [fact] + dims
    trees = [datagen.star_fact_predicate()] + datagen.star_dim_predicates()
    caps = [0] + [d.nrows for d in dims]
    got = run_both(sel, ctx, tables, trees, caps, 1000, 0.05)
    assert [g["decision"] for g in got] == ["probe", "reverted", "reverted", "reverted", "pushed"]
    assert [g["order"] for g in got] == [None, 3, 2, 1, 0]


def test_spd_rejects_bad_input(sel, ctx):
    rng = np.random.default_rng(72_000)
    a = sel.device_table(ctx, datagen.random_table(rng, 3000, null_rate=0.0))
    b = sel.device_table(ctx, datagen.random_table(rng, 2000, null_rate=0.0))
    pb = ctx.program(b, ("cmp", 0, ">", 0))
    with pytest.raises(sel.SelError):
        ctx.select_pushdown([])
    with pytest.raises(sel.SelError):
        ctx.select_pushdown([(a, None, None), (b, pb, None)], max_selectivity=float("nan"))
    with pytest.raises(sel.SelError):   # a program bound to another table
        ctx.select_pushdown([(a, pb, None), (b, None, None)])
    # a NULL buffer with no capacity: the pushed relation needs none if empty
    pe = ctx.program(b, ("cmp", 0, ">", 10 ** 6))
    r = ctx.select_pushdown([(a, None, None), (b, pe, None)])
    assert r[1]["decision"] == "pushed" and r[1]["count"] == 0


def test_factor_counts_match_oracle(sel, ctx):
    """A selection's conjunct counts and its own count, from one batched
    launch, equal the oracle's (as multisets: the compiler may reorder
    operands), and so does the independence estimate built from them; on
    random programs with NULLs and on the fact-table predicate."""
    rng = np.random.default_rng(73_000)
    t = datagen.random_table(rng, 100_003, grid=False, null_rate=0.2)
    dt = sel.device_table(ctx, t)
    trees = [sqlite_ref.clamp_literals(datagen.random_tree(rng, t, grid=False)) for _ in range(12)]
    for _ in range(3):
        trees.append(("and",) + tuple(sqlite_ref.clamp_literals(
            datagen.random_tree(rng, t, max_depth=3, max_leaves=3, grid=False)) for _ in range(5)))
    for tree in trees:
        prog = ctx.program(dt, tree)
        c, fc = ctx.factor_counts(dt, prog)
        wc, wfc = oracle.factor_counts(t, tree)
        assert c == wc and sorted(fc) == sorted(wfc), tree
        assert ctx.independence_estimate(t.nrows, fc) == pytest.approx(
            oracle.independence_estimate(t.nrows, wfc), rel=1e-12)
    f = datagen.cfg2(n=2_000_003, threads=16)
    df = sel.device_table(ctx, f)
    tree = datagen.cfg2_predicate()
    c, fc = ctx.factor_counts(df, ctx.program(df, tree))
    wc, wfc = oracle.factor_counts(f, tree, threads=16)
    assert c == wc and len(fc) == 4 and sorted(fc) == sorted(wfc)


def test_star_plan_from_exact_counts(sel, ctx):
    """The join order of a star query from the GPU's exact dimension counts
    equals the oracle's cheapest order from its own counts, and the formula's
    final size lands near the exact star count (independent uniform keys)."""
    say("star plan: generating")
    dims = datagen.star_dims()
    fact = datagen.star_fact(10_000_000, threads=16)
    preds = datagen.star_dim_predicates()
    ddims = [sel.device_table(ctx, d) for d in dims]
    dfact = sel.device_table(ctx, fact)
    counts, bms = [], []
    for d, dd, p in zip(dims, ddims, preds):
        c = ctx.count(dd, ctx.program(dd, p))
        assert c == oracle.Oracle(d).count(p)
        counts.append(c)
        bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
        st, c2 = ctx.pushdown_keybitmap(dd, 0, 0, ctx.program(dd, p), bm, d.nrows)
        assert st == sel.SEL_OK and c2 == c
        bms.append(bm)
    rows = [d.nrows for d in dims]
    order, cost, inter = sel.star_plan(fact.nrows, rows, counts)
    want_order, want_cost = oracle.best_star_plan(fact.nrows, rows, counts)
    assert order == want_order and cost == pytest.approx(want_cost, rel=1e-12)
    exact = ctx.star_count(dfact, [0, 1, 2, 3], bms, rows)
    assert exact > 0 and 1 / 1.5 < inter[-1] / exact < 1.5
