"""GPU: batched counts (one persistent launch, eager and graph-replayed)
equal the plain counts and the oracle, bit-exactly.  Every test runs three
times: with the lookup-table kernel taking every program in conjunctive
form (SEL_BATCH_KERNEL=lut; the rest, e.g. with IS UNKNOWN, in the
leaf-major kernel of the same launch), with the leaf-major kernel alone
(SEL_BATCH_KERNEL=leaf), and with the default split by chunk length."""
import os

import numpy as np
import pytest

import datagen
import oracle
from tests import sqlite_ref
from tests.gpu_common import UINT64_MAX, as_u32, ids_tensor, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True, params=["lut", "leaf", "default"])
def batch_kernel(request):
    old = os.environ.get("SEL_BATCH_KERNEL")
    if request.param == "default":
        os.environ.pop("SEL_BATCH_KERNEL", None)
    else:
        os.environ["SEL_BATCH_KERNEL"] = request.param
    say(f"batch kernel: {request.param}")
    yield request.param
    if old is None:
        os.environ.pop("SEL_BATCH_KERNEL", None)
    else:
        os.environ["SEL_BATCH_KERNEL"] = old


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
def setup(sel, ctx):
    """Four tables of uneven size (10k .. 3M rows, partial last tiles) and the
    64 candidate programs of the batching workload."""
    say("batch: generating tables")
    rows = (10_000, 200_003, 1_000_000, 3_000_001)
    tables = datagen.cfg3_tables(rows=rows)
    dts = [sel.device_table(ctx, t) for t in tables]
    progs = datagen.cfg3_programs()
    pairs = [(dts[t], ctx.program(dts[t], tree)) for t, tree in progs]
    want = [oracle.Oracle(tables[t]).count(tree, threads=8) for t, tree in progs]
    return tables, dts, progs, pairs, want


def test_batch_equals_plain_and_oracle(sel, ctx, setup):
    tables, dts, progs, pairs, want = setup
    plain = [ctx.count(t, p) for t, p in pairs]
    assert plain == want
    got = ctx.count_batch(pairs)
    assert got == want
    # selectivities span orders of magnitude
    sel_ = [w / tables[t].nrows for (t, _), w in zip(progs, want)]
    assert min(sel_) < 1e-3 and max(sel_) > 0.1


def test_batch_subsets_and_repeats(sel, ctx, setup):
    tables, dts, progs, pairs, want = setup
    rng = np.random.default_rng(4)
    for _ in range(5):
        idx = [int(i) for i in rng.integers(0, len(pairs), int(rng.integers(1, 40)))]
        got = ctx.count_batch([pairs[i] for i in idx])
        assert got == [want[i] for i in idx]
    # a single pair, and one table only
    assert ctx.count_batch([pairs[5]]) == [want[5]]
    only3 = [i for i, (t, _) in enumerate(progs) if t == 3]
    assert ctx.count_batch([pairs[i] for i in only3]) == [want[i] for i in only3]


def test_graph_replay(sel, ctx, setup):
    """Replay several times with the program's own eager work between the
    replays; every replay equals the eager result."""
    tables, dts, progs, pairs, want = setup
    b = ctx.batch(pairs)
    for r in range(4):
        assert b.run() == want, f"replay {r}"
        # eager work on the same context in between
        assert ctx.count_batch(pairs[:7]) == want[:7]
        assert ctx.count(*pairs[r]) == want[r]
    b.destroy()


def test_graph_descriptor_update(sel, ctx, setup):
    """Swapping a program rewrites the descriptor only; the replay then
    equals a fresh eager batch."""
    tables, dts, progs, pairs, want = setup
    b = ctx.batch(pairs)
    assert b.run() == want
    t3 = [i for i, (t, _) in enumerate(progs) if t == 3]
    i = t3[0]
    new_tree = datagen.cfg2_predicate(100, 900)
    newp = ctx.program(dts[3], new_tree)
    b.set_program(i, newp)
    w2 = list(want)
    w2[i] = oracle.Oracle(tables[3]).count(new_tree, threads=8)
    for _ in range(3):
        assert b.run() == w2
    pairs2 = list(pairs)
    pairs2[i] = (dts[3], newp)
    assert ctx.count_batch(pairs2) == w2
    with pytest.raises(sel.SelError):
        b.set_program(i, pairs[0][1])     # a program of another table
    b.destroy()


def test_batch_empty_and_tiny_tables(sel, ctx):
    t0 = datagen.cfg1(0, seed=1)
    t1 = datagen.cfg1(1, seed=2)
    t2 = datagen.cfg1(2049, seed=3)
    dts = [sel.device_table(ctx, t) for t in (t0, t1, t2)]
    tree = ("cmp", 0, "<", 5000)
    pairs = [(d, ctx.program(d, tree)) for d in dts]
    want = [oracle.Oracle(t).count(tree) for t in (t0, t1, t2)]
    assert ctx.count_batch(pairs) == want
    assert ctx.count_batch(pairs[:1]) == [0]
    b = ctx.batch(pairs)
    assert b.run() == want
    b.destroy()


def test_batch_rejects_bad_input(sel, ctx, setup):
    tables, dts, progs, pairs, want = setup
    with pytest.raises(sel.SelError):
        ctx.count_batch([(dts[0], pairs[-1][1])])   # program of another table
    with pytest.raises(sel.SelError):
        ctx.count_batch([])


def test_rows_per_lane_keeps_results(sel, ctx, setup):
    """The lookup-table kernel with four or eight rows per lane per segment
    gives the same exact counts."""
    tables, dts, progs, pairs, want = setup
    try:
        for rows in (4, 8):
            ctx.set_launch(256, 0, rows_per_lane=rows)
            assert ctx.count_batch(pairs) == want, rows
        with pytest.raises(sel.SelError):
            ctx.set_launch(256, 0, rows_per_lane=5)
    finally:
        ctx.set_launch(None)


def test_autotune_keeps_results(sel, ctx, setup, tmp_path):
    """Tuning changes launch shapes only: counts stay exact, and the tuned
    table survives a save/load round trip into a fresh context."""
    tables, dts, progs, pairs, want = setup
    cfg, ms = ctx.autotune(*pairs[-1], with_mask=False, reps=2)
    block, grid = cfg.block, cfg.grid
    assert block in (64, 128, 256) and grid > 0 and ms > 0
    ctx.autotune(*pairs[-1], with_mask=True, reps=2)
    bcfg, bms = ctx.autotune_batch(pairs, reps=1)
    bb, bg = bcfg.block, bcfg.grid
    assert bb in (64, 128, 256, 512, 768) and bg > 0
    assert ctx.tune_entries >= 3
    assert ctx.count(*pairs[-1]) == want[-1]
    # the tuned mask-pass shape still gives the oracle's ids
    t, tree = progs[-1]
    out = ids_tensor(want[-1], torch)
    st, cnt = ctx.pushdown_rowids(*pairs[-1], UINT64_MAX, out)
    assert (st, cnt) == (sel.SEL_OK, want[-1])
    np.testing.assert_array_equal(as_u32(out)[:cnt], oracle.Oracle(tables[t]).rowids(tree))
    assert ctx.count_batch(pairs) == want
    path = tmp_path / "tune.txt"
    ctx.tune_save(path)
    c2 = sel.Context(0)
    c2.tune_load(path)
    assert c2.tune_entries == ctx.tune_entries
    c2.close()


@pytest.mark.parametrize("n", [1, 2049, 100_003])
def test_batch_random_programs(sel, ctx, n):
    """Random programs (every operator, NULLs, value lists, code sets) on two
    random tables of ragged size, batched together: enough programs that the
    batch splits into several passes per table.  Each count equals the plain
    count and the oracle."""
    say(f"batch random n={n}")
    rng = np.random.default_rng(20_000 + n)
    ts = [datagen.random_table(rng, n, grid=True, null_rate=0.3),
          datagen.random_table(rng, n + 4097, grid=False, null_rate=0.1)]
    dts = [sel.device_table(ctx, t) for t in ts]
    orcs = [oracle.Oracle(t) for t in ts]
    trees = []
    for k in range(90):
        ti = k % 2
        trees.append((ti, sqlite_ref.clamp_literals(datagen.random_tree(rng, ts[ti]))))
    pairs = [(dts[ti], ctx.program(dts[ti], tree)) for ti, tree in trees]
    want = [orcs[ti].count(tree) for ti, tree in trees]
    assert ctx.count_batch(pairs) == want
    assert [ctx.count(*p) for p in pairs[:10]] == want[:10]
    # the same program several times, and a replayed graph of the set
    assert ctx.count_batch([pairs[3]] * 5 + pairs[:4]) == [want[3]] * 5 + want[:4]
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()


@pytest.mark.parametrize("nstar", [12, 20])
def test_batch_star_programs(sel, ctx, nstar):
    """Star semi-join programs in one batch, over dimensions that take every
    lookup route: with 12 programs (2-byte entries) an LDS table (2556 keys)
    and device-memory tables (30k, 600k and 9M keys, the largest read only
    where the earlier probes leave rows); with 20 (4-byte entries) the 600k
    table is read only where guards hold and the 9M keys are probed in the
    dimension bitmaps themselves.  With fact-side predicates, a plain fact
    program and a program used twice (no guard)."""
    sizes = (2556, 30_000, 600_000, 9_000_000)
    say("batch star: generating dimensions and fact")
    dims = datagen.star_dims(seed=42, sizes=sizes)
    fact = datagen.star_fact(1_000_003, dim_rows=sizes)
    ddims = [sel.device_table(ctx, d) for d in dims]
    dfact = sel.device_table(ctx, fact)
    ofact = oracle.Oracle(fact)
    fp = datagen.star_fact_predicate()
    progs, want, keep = [], [], []
    for k, combo in enumerate(datagen.star_dim_programs(7, nstar, dims)):
        bms_gpu, bms_cpu = [], []
        for d, dt, p in zip(dims, ddims, combo):
            bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
            st, _ = ctx.pushdown_keybitmap(dt, 0, 0, ctx.program(dt, p), bm, d.nrows)
            assert st == sel.SEL_OK
            ost, _, owords = oracle.Oracle(d).keybitmap(p, 0, 0, d.nrows)
            assert ost == 0
            bms_gpu.append(bm)
            bms_cpu.append(owords)
        keep.append(bms_gpu)
        pred = ctx.program(dfact, fp) if k % 3 == 2 else None
        progs.append(ctx.star_program(dfact, [0, 1, 2, 3], bms_gpu, list(sizes), pred))
        want.append(ofact.star_count([0, 1, 2, 3], bms_cpu, list(sizes),
                                     fp if pred is not None else None, threads=8))
    progs.append(ctx.program(dfact, fp))
    want.append(ofact.count(fp, threads=8))
    progs.append(progs[0])
    want.append(want[0])
    pairs = [(dfact, p) for p in progs]
    assert [ctx.count(*p) for p in pairs] == want
    assert ctx.count_batch(pairs) == want
    assert ctx.count_batch(pairs[:5]) == want[:5]
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()


def _nulls(rng, n, rate):
    """Validity words (bit i % 32 of word i / 32 = not NULL) and NULL count."""
    isnull = rng.random(n) < rate
    bits = np.packbits((~isnull).astype(np.uint8), bitorder="little")
    buf = np.zeros((n + 31) // 32 * 4, dtype=np.uint8)
    buf[: bits.size] = bits
    return buf.view(np.uint32).copy(), int(isnull.sum())


@pytest.mark.parametrize("k,span", [(6, 50_000), (12, 50_000), (24, 50_000), (12, 500_000),
                                    (24, 500_000)])
def test_batch_table_widths(sel, ctx, k, span):
    """k programs over the same two narrow columns, so that one lookup table
    per column serves all their leaves, with entries of 1, 2 or 4 bytes (up
    to 8, 16 or 32 leaves): in LDS for an int8 column with NULLs, and in
    device memory for an int32 code column of `span` values (code sets of a
    compiled program are at most 512k bits; the larger guarded tables and
    probes are reached by the star programs).  Every fourth program puts its
    int8 test in an OR, which keeps that leaf out of the accumulator.
    Counts equal the oracle and the plain counts, eager and replayed."""
    say(f"batch table widths k={k} span={span}")
    rng = np.random.default_rng(31_000 + 7 * k + span)
    n = 200_003
    t = datagen.Table("widths", n)
    t.columns.append(datagen.Column("a", "i32", rng.integers(0, span, n).astype(np.int32),
                                    dict_card=span))
    vb, nb = _nulls(rng, n, 0.1)
    t.columns.append(datagen.Column("b", "i8", rng.integers(-100, 101, n).astype(np.int8),
                                    valid=vb, null_count=nb))
    vc, nc = _nulls(rng, n, 0.05)
    t.columns.append(datagen.Column("c", "i64", rng.integers(0, 1_000_000, n).astype(np.int64),
                                    valid=vc, null_count=nc))
    nw = (span + 31) // 32
    trees = []
    for i in range(k):
        lo = int(rng.integers(-100, 60))
        hi = lo + int(rng.integers(5, 80))
        words = rng.integers(0, 2**32, nw, dtype=np.uint32)
        for _ in range(int(rng.integers(0, 3))):   # code density 1/2, 1/4 or 1/8
            words &= rng.integers(0, 2**32, nw, dtype=np.uint32)
        thr = int(rng.integers(0, 1_000_000))
        if i % 4 == 3:
            trees.append(("and", ("or", ("between", 1, lo, hi), ("cmp", 2, "<", thr)),
                          ("codeset", 0, span, words)))
        else:
            trees.append(("and", ("between", 1, lo, hi), ("codeset", 0, span, words),
                          ("cmp", 2, ">=", thr)))
    dt = sel.device_table(ctx, t)
    pairs = [(dt, ctx.program(dt, tree)) for tree in trees]
    orc = oracle.Oracle(t)
    want = [orc.count(tree) for tree in trees]
    assert ctx.count_batch(pairs) == want
    assert [ctx.count(*p) for p in pairs[:4]] == want[:4]
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()


def test_batch_wide_program(sel, ctx):
    """A program with more leaf and validity words than a shared pass packs
    (an OR of 32 int64 range tests over 12 nullable columns: 44 slots) runs
    in a pass of its own with smaller workgroups; batched with ordinary
    programs, alone, and replayed, every count equals the oracle."""
    say("batch wide program")
    rng = np.random.default_rng(41_000)
    n = 100_003
    t = datagen.Table("wide", n)
    for c in range(12):
        v, nn = _nulls(rng, n, 0.05)
        t.columns.append(datagen.Column(f"c{c}", "i64", rng.integers(0, 10**6, n).astype(np.int64),
                                        valid=v, null_count=nn))
    leaves = []
    for i in range(32):
        lo = int(rng.integers(0, 10**6 - 10**4))
        leaves.append(("between", i % 12, lo, lo + 10**4))
    trees = [("or", *leaves)]
    for i in range(6):
        lo = int(rng.integers(0, 10**6 - 10**5))
        trees.append(("and", ("cmp", i, ">=", int(rng.integers(0, 10**6))),
                      ("between", i + 1, lo, lo + 10**5)))
    dt = sel.device_table(ctx, t)
    pairs = [(dt, ctx.program(dt, tree)) for tree in trees]
    orc = oracle.Oracle(t)
    want = [orc.count(tree) for tree in trees]
    assert ctx.count_batch(pairs) == want
    assert ctx.count_batch(pairs[:1]) == want[:1]
    assert ctx.count_batch(pairs[1:]) == want[1:]
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()


def test_batch_full_size(sel, ctx):
    """The batching workload at its full sizes (10k / 2M / 60M / 300M rows,
    64 programs) in the default launch shape and as a graph: every count
    equals the threaded oracle."""
    say("batch full: generating tables")
    tables = datagen.cfg3_tables(threads=16)
    dts = [sel.device_table(ctx, t) for t in tables]
    progs = datagen.cfg3_programs()
    pairs = [(dts[t], ctx.program(dts[t], tree)) for t, tree in progs]
    say("batch full: GPU batch")
    got = ctx.count_batch(pairs)
    b = ctx.batch(pairs)
    got_graph = b.run()
    b.destroy()
    say("batch full: oracle")
    orcs = [oracle.Oracle(t) for t in tables]
    want = [orcs[t].count(tree, threads=16) for t, tree in progs]
    assert got == want
    assert got_graph == want
    del dts, pairs
    torch.cuda.empty_cache()


def test_batch_conjunction_shapes(sel, ctx):
    """Conjunctions that take every fast path of the batch planner, on a
    table whose columns all have NULLs: direct factors (into the program's
    accumulator, bitmap ones guarded), OR groups of narrow tests (into one
    word), int64 leaves and OR groups with an int64 leaf (slots), evaluated
    as lists of TRUE words; and the same shapes under NOT, which keeps the
    three-valued interpreter.  Counts equal the oracle, eager and replayed."""
    rng = np.random.default_rng(42_000)
    n = 150_011
    t = datagen.Table("shapes", n)
    for name, ty, lo, hi in (("a", "i8", -50, 50), ("b", "i16", -3000, 3000),
                             ("c", "i32", 0, 20_000), ("d", "i64", -10**9, 10**9),
                             ("e", "i32", 0, 4_000)):
        v, nn = _nulls(rng, n, 0.08)
        t.columns.append(datagen.Column(name, ty, rng.integers(lo, hi, n).astype(
            {"i8": np.int8, "i16": np.int16, "i32": np.int32, "i64": np.int64}[ty]),
            valid=v, null_count=nn, dict_card=4_000 if name == "e" else 0))

    def leaf(col):
        if col == 0:
            x = int(rng.integers(-50, 40))
            return ("between", 0, x, x + int(rng.integers(1, 60)))
        if col == 1:
            return ("cmp", 1, str(rng.choice(["<", ">=", "<>"])), int(rng.integers(-3000, 3000)))
        if col == 2:
            return ("in", 2, tuple(int(v) for v in rng.choice(20_000, 40, replace=False)))
        if col == 3:
            return ("cmp", 3, str(rng.choice([">=", "<"])), int(rng.integers(-10**9, 10**9)))
        w = rng.integers(0, 2**32, 125, dtype=np.uint32) & rng.integers(0, 2**32, 125, dtype=np.uint32)
        return ("codeset", 4, 4_000, w)

    trees = []
    for k in range(40):
        factors = [leaf(int(rng.integers(0, 5))) for _ in range(int(rng.integers(1, 4)))]
        factors.append(("or",) + tuple(leaf(int(c)) for c in rng.choice([0, 1, 2, 4], 2, replace=False)))
        if k % 2:
            factors.append(("or", leaf(3), leaf(int(rng.integers(0, 3)))))
        tree = ("and",) + tuple(factors)
        trees.append(("not", tree) if k % 5 == 4 else tree)
    dt = sel.device_table(ctx, t)
    pairs = [(dt, ctx.program(dt, tree)) for tree in trees]
    orc = oracle.Oracle(t)
    want = [orc.count(tree) for tree in trees]
    assert ctx.count_batch(pairs) == want
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()


@pytest.mark.parametrize("nb", [1, 3, 4, 5, 8, 13, 16, 17, 31])
def test_batch_rank_bounds(sel, ctx, nb):
    """A pass whose int64 and int32 columns are looked up by rank (value
    ranges too wide for a direct window) with nb distinct bounds each, from
    one bound to a whole block of eight and past it.  The values include
    both ends of each type, every bound itself and NULLs; counts equal the
    oracle."""
    say(f"batch rank bounds nb={nb}")
    rng = np.random.default_rng(43_000 + nb)
    n = 70_001
    i64 = np.iinfo(np.int64)
    i32 = np.iinfo(np.int32)
    b64 = np.sort(rng.choice(rng.integers(-10**15, 10**15, 4 * nb), nb, replace=False)).astype(np.int64)
    b32 = np.sort(rng.choice(rng.integers(i32.min, i32.max, 4 * nb, dtype=np.int64), nb,
                             replace=False)).astype(np.int32)
    x64 = rng.integers(-2 * 10**15, 2 * 10**15, n).astype(np.int64)
    x32 = rng.integers(i32.min, i32.max, n, dtype=np.int64).astype(np.int32)
    k = np.arange(n)
    x64[k % 7 == 0] = b64[(k[k % 7 == 0] // 7) % nb]
    x32[k % 5 == 0] = b32[(k[k % 5 == 0] // 5) % nb]
    x64[:6] = [i64.min, i64.max, i64.min + 1, i64.max - 1, 0, -1]
    x32[:4] = [i32.min, i32.max, i32.min + 1, i32.max - 1]
    t = datagen.Table("ranks", n)
    for name, x in (("w", x64), ("v", x32)):
        v, nn = _nulls(rng, n, 0.1)
        t.columns.append(datagen.Column(name, "i64" if x.dtype == np.int64 else "i32", x,
                                        valid=v, null_count=nn))
    trees = []
    for j in range(nb):
        # one bound per leaf: x >= b_j, or x < b_j; the second column's
        # leaf keeps each program two-column
        op = ">=" if j % 2 == 0 else "<"
        trees.append(("and", ("cmp", 0, op, int(b64[j])), ("cmp", 1, "<" if j % 3 else ">=", int(b32[j]))))
    trees.append(("cmp", 0, ">=", int(b64[-1])))
    trees.append(("or", ("cmp", 0, "<", int(b64[0])), ("cmp", 1, ">=", int(b32[-1]))))
    dt = sel.device_table(ctx, t)
    pairs = [(dt, ctx.program(dt, tree)) for tree in trees]
    orc = oracle.Oracle(t)
    want = [orc.count(tree) for tree in trees]
    assert ctx.count_batch(pairs) == want
    b = ctx.batch(pairs)
    for _ in range(2):
        assert b.run() == want
    b.destroy()
