"""GPU parity: libsel's HIP path (through the C ABI) against the CPU oracle,
bit-exact on every count, every row-id array and every key bitmap."""
import numpy as np
import pytest

import datagen
import oracle
from tests import sqlite_ref
from tests.gpu_common import UINT64_MAX, as_u32, ids_tensor, say

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


def gpu_ids(sel, ctx, dt, prog, n_hint):
    out = ids_tensor(n_hint, torch)
    st, cnt = ctx.pushdown_rowids(dt, prog, UINT64_MAX, out)
    assert st == sel.SEL_OK
    return cnt, as_u32(out)[:cnt]


def check_tree(sel, ctx, dt, orc, tree, ids=True):
    prog = ctx.program(dt, tree)
    want = orc.count(tree)
    got = ctx.count(dt, prog)
    assert got == want, (tree, prog.listing)
    if ids:
        cnt, got_ids = gpu_ids(sel, ctx, dt, prog, want)
        assert cnt == want
        np.testing.assert_array_equal(got_ids, orc.rowids(tree))
    return want


def test_cfg1_count_and_ids(sel, ctx):
    say("cfg1: 1M rows x 3 int32, P1")
    t = datagen.cfg1()
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    c = check_tree(sel, ctx, dt, orc, datagen.cfg1_predicate())
    assert 26_000 < c < 28_000


@pytest.mark.parametrize("n", [0, 1, 3, 63, 64, 65, 255, 256, 257, 2047, 2048, 2049,
                               4096 + 5, 8192, 3 * 2048 + 1000, 100_003])
def test_ragged_sizes_random_programs(sel, ctx, n):
    say(f"ragged n={n}")
    rng = np.random.default_rng(10_000 + n)
    t = datagen.random_table(rng, n, grid=True, null_rate=0.3)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    for k in range(12):
        tree = sqlite_ref.clamp_literals(datagen.random_tree(rng, t))
        check_tree(sel, ctx, dt, orc, tree)


def test_mask_lane_patterns(sel, ctx):
    """Row-id materialisation where the TRUE rows sit in chosen lanes of each
    2048-row tile (lane L of a tile holds rows 256 j + 4 L + i): only the
    first or the last lane, alternate lanes, the upper half, every lane, no
    lane, and a mix that changes from tile to tile (first and last lane,
    a whole tile, one row of lane 31, an empty tile), on a ragged table.
    The mask pass writes only a tile's words that hold a TRUE row, packed in
    lane order, and the compaction places each by its lane's rank."""
    n = 2048 * 37 + 777
    r = np.arange(n, dtype=np.int64)
    t = datagen.Table("lanes", n)
    t.columns.append(datagen.Column("lane", "i8", ((r % 256) // 4).astype(np.int8)))
    t.columns.append(datagen.Column("tmod", "i8", ((r // 2048) % 4).astype(np.int8)))
    t.columns.append(datagen.Column("step", "i8", ((r % 2048) // 256).astype(np.int8)))
    t.columns.append(datagen.Column("i", "i8", (r % 4).astype(np.int8)))
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    trees = [
        ("cmp", 0, "=", 63),
        ("cmp", 0, "=", 0),
        ("in", 0, tuple(range(0, 64, 2))),
        ("and", ("cmp", 0, ">=", 32), ("cmp", 1, "<>", 2)),
        ("cmp", 0, ">=", 0),
        ("cmp", 0, ">", 63),
        ("or", ("and", ("cmp", 1, "=", 0), ("in", 0, (0, 63))),
               ("cmp", 1, "=", 1),
               ("and", ("cmp", 1, "=", 2), ("cmp", 0, "=", 31), ("cmp", 2, "=", 7), ("cmp", 3, "=", 3))),
    ]
    for tree in trees:
        say(f"lane pattern {tree}")
        check_tree(sel, ctx, dt, orc, tree)


def test_mask_sparse_lane_patterns(sel, ctx):
    """Row-id materialisation of tiles where no lane holds more than two TRUE
    rows (the compaction places them by walking each lane's set bits): one
    row per lane at a step and position that vary with the lane, two rows of
    one lane in the same 4-row group, two rows in different steps, and tiles
    where one lane holds three rows (the general path) beside lanes with
    one; the patterns alternate with empty and full tiles, on a ragged
    table."""
    n = 2048 * 29 + 1311
    r = np.arange(n, dtype=np.int64)
    lane, step, i = (r % 256) // 4, (r % 2048) // 256, r % 4
    tmod = (r // 2048) % 4
    l8 = lane % 8
    t = datagen.Table("sparse_lanes", n)
    cols = {
        "one": (step == l8) & (i == lane % 4),
        "same_group": (step == l8) & ((i == 1) | (i == 3)),
        "two_steps": (i == 0) & ((step == l8) | (step == (l8 + 3) % 8)),
        "three": ((lane == 5) & (step < 3) & (i == 0)) | ((lane != 5) & (step == 2) & (i == 1)),
        "tmod": tmod,
    }
    for name, v in cols.items():
        t.columns.append(datagen.Column(name, "i8", v.astype(np.int8)))
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    trees = [
        ("cmp", 0, "=", 1),
        ("cmp", 1, "=", 1),
        ("cmp", 2, "=", 1),
        ("cmp", 3, "=", 1),
        ("or", ("and", ("cmp", 4, "=", 0), ("cmp", 1, "=", 1)),
               ("and", ("cmp", 4, "=", 1), ("cmp", 3, "=", 1)),
               ("and", ("cmp", 4, "=", 2), ("cmp", 2, "=", 1)),
               ("and", ("cmp", 4, "=", 3), ("cmp", 0, "=", 0))),
        ("and", ("cmp", 4, "<>", 1), ("or", ("cmp", 0, "=", 1), ("cmp", 2, "=", 1))),
    ]
    for tree in trees:
        say(f"sparse lane pattern {tree}")
        check_tree(sel, ctx, dt, orc, tree)


def test_random_programs_small_ranges(sel, ctx):
    """Values in a small range so that comparisons split rows evenly."""
    rng = np.random.default_rng(77)
    t = datagen.random_table(rng, 50_000, grid=False, null_rate=0.2)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    for k in range(60):
        tree = datagen.random_tree(rng, t, grid=False)
        check_tree(sel, ctx, dt, orc, tree, ids=(k % 3 == 0))


@pytest.mark.parametrize("k", [10, 100, 1000, 3000])
def test_sparse_in_lists(sel, ctx, k):
    """IN lists too sparse for a bitmap (the compiler keeps them as sorted
    lists): k values drawn from the column plus as many absent ones, on an
    int64 log-normal column with NULLs, an int32 and an int8 column, over a
    ragged 1 000 003-row table; lists up to 4095 values are searched in the
    scan's LDS copy, the 6000-value lists in device memory.
    Counts and ids equal the oracle; alone, under NOT and inside an AND."""
    say(f"sparse IN lists k={k}")
    rng = np.random.default_rng(90_000 + k)
    t = datagen.cfg2(n=1_000_003, seed=91)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    price = t.col("price").data
    date = t.col("date").data

    def pick(col, absent_lo, absent_hi):
        present = rng.choice(col, k, replace=False)
        absent = rng.integers(absent_lo, absent_hi, k)
        return tuple(int(v) for v in np.concatenate([present, absent]))

    trees = [("in", 3, pick(price, 10**7, 10**8)),
             ("not", ("in", 3, pick(price, -10**6, 0))),
             ("in", 0, pick(date, 3000, 10**6)),
             ("and", ("in", 3, pick(price, 10**7, 10**8)), ("between", 1, 5, 40)),
             ("in", 1, tuple(int(v) for v in rng.integers(-128, 128, min(k, 200))))]
    for tree in trees:
        check_tree(sel, ctx, dt, orc, tree, ids=True)


def test_kleene_single_rows(sel, ctx):
    """Every (a, b) in {T, U, F}^2 on one-row tables, through the GPU."""
    from tests.oracle_pins import GOLDEN, SYM, _leaf_table
    import os
    vals = {"T": 1, "F": 0, "U": None}
    with open(os.path.join(GOLDEN, "kleene_k3.txt")) as f:
        rows = [l.split("#")[0].split() for l in f if l.split("#")[0].strip()]
    for op, a, b, res in rows:
        t = _leaf_table([vals[a]])
        leaf0, leaf1 = ("cmp", 0, "=", 1), ("cmp", 1, "=", 1)
        if b == "-":
            tree = ("not", leaf0) if op == "NOT" else ("isunknown", leaf0)
        else:
            t.columns[1].data[:] = 0 if vals[b] is None else vals[b]
            t.columns[1].valid[:] = 0 if vals[b] is None else 1
            tree = (op.lower(), leaf0, leaf1)
        dt = sel.device_table(ctx, t)
        got = ctx.count(dt, ctx.program(dt, tree))
        assert got == (1 if SYM[res] == oracle.T else 0), (op, a, b)


def test_cfg2_small(sel, ctx):
    say("cfg2 at 2M rows")
    t = datagen.cfg2(n=2_000_000)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    check_tree(sel, ctx, dt, orc, datagen.cfg2_predicate())
    for lo, hi in [(0, 0), (0, 2556), (100, 99), (2000, 2600), (-5, 3)]:
        check_tree(sel, ctx, dt, orc, datagen.cfg2_predicate(lo, hi))
    # leaf-count sweep (1..8 leaves) and NULL handling on price
    leaves = [("between", 0, 365, 729), ("cmp", 1, "<", 25), ("between", 2, 5, 7),
              ("cmp", 3, ">=", 20000), ("in", 5, tuple(range(0, 20, 2))),
              ("codeset", 6, 4500, datagen.cfg2_like_bitmap()), ("cmp", 4, "<>", 0),
              ("isnull", 3)]
    for k in range(1, len(leaves) + 1):
        check_tree(sel, ctx, dt, orc, ("and", *leaves[:k]) if k > 1 else leaves[0], ids=(k % 2 == 0))
    check_tree(sel, ctx, dt, orc, ("isunknown", ("cmp", 3, ">=", 20000)))
    check_tree(sel, ctx, dt, orc, ("not", ("cmp", 3, "<", 20000)))


def test_limits_and_capacity(sel, ctx):
    """Algorithm 1: count > max_rows aborts with nothing written."""
    t = datagen.cfg1(200_000, seed=5)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    tree = datagen.cfg1_predicate()
    prog = ctx.program(dt, tree)
    c = orc.count(tree)
    ids = orc.rowids(tree)
    out = ids_tensor(c + 10, torch)
    st, cnt = ctx.pushdown_rowids(dt, prog, c - 1, out)
    assert (st, cnt) == (sel.SEL_OVER_LIMIT, c)
    assert np.all(as_u32(out) == 0xDEADBEEF)
    st, cnt = ctx.pushdown_rowids(dt, prog, c + 10, out, cap=c - 1)
    assert (st, cnt) == (sel.SEL_E_CAPACITY, c)
    assert np.all(as_u32(out) == 0xDEADBEEF)
    st, cnt = ctx.pushdown_rowids(dt, prog, c, out)
    assert (st, cnt) == (sel.SEL_OK, c)
    np.testing.assert_array_equal(as_u32(out)[:c], ids)
    assert np.all(as_u32(out)[c:] == 0xDEADBEEF)
    st, cnt = ctx.pushdown_rowids(dt, prog, sel.max_rows(t.nrows, c / t.nrows), out)
    assert st == sel.SEL_OK
    # max_rows = 0 with an empty result is accepted (strict >)
    p0 = ctx.program(dt, ("false",))
    assert ctx.pushdown_rowids(dt, p0, 0, out) == (sel.SEL_OK, 0)


def test_launch_shapes_agree(sel, ctx):
    """Results do not depend on block size or grid size (ordered compaction
    and exact counts under any workgroup interleaving)."""
    t = datagen.cfg2(n=1_000_003, seed=12)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    tree = datagen.cfg2_predicate(0, 1200)
    want = orc.count(tree)
    want_ids = orc.rowids(tree)
    prog = ctx.program(dt, tree)
    try:
        for block, grid in [(64, 1), (64, 7), (128, 33), (256, 0), (256, 3), (128, 10_000)]:
            ctx.set_launch(block, grid)
            assert ctx.count(dt, prog) == want, (block, grid)
            cnt, ids = gpu_ids(sel, ctx, dt, prog, want)
            assert cnt == want
            np.testing.assert_array_equal(ids, want_ids)
        # the tuner's other knobs: cached loads, runs of tiles per wave step
        # (the last run cut at the table's end), LDS staging limited or off
        for block, grid, cached, tps, stage in [(256, 0, 1, 1, 0), (64, 7, 0, 4, 0), (128, 33, 0, 2, 1),
                                                (256, 3, 1, 4, 2048), (256, 0, 0, 2, 1)]:
            ctx.set_launch(block, grid, cached=cached, tiles_per_step=tps, stage_words=stage)
            assert ctx.count(dt, prog) == want, (block, grid, cached, tps, stage)
            cnt, ids = gpu_ids(sel, ctx, dt, prog, want)
            assert cnt == want
            np.testing.assert_array_equal(ids, want_ids)
        with pytest.raises(sel.SelError):
            ctx.set_launch(256, 0, tiles_per_step=3)
    finally:
        ctx.set_launch(None)


def test_async_count(sel, ctx):
    t = datagen.cfg1(300_000, seed=8)
    dt = sel.device_table(ctx, t)
    tree = datagen.cfg1_predicate()
    prog = ctx.program(dt, tree)
    out = torch.zeros(4, dtype=torch.int64, device="cuda")
    for k in range(4):
        ctx.count_async(dt, prog, out.data_ptr() + 8 * k)
    torch.cuda.synchronize()
    want = oracle.Oracle(t).count(tree)
    assert out.cpu().tolist() == [want] * 4


def star_setup(sel, ctx, fact_rows, dim_rows):
    dims = datagen.star_dims(sizes=dim_rows)
    preds = datagen.star_dim_predicates()
    fact = datagen.star_fact(fact_rows, dim_rows=dim_rows)
    return dims, preds, fact


def test_keybitmaps_and_star(sel, ctx):
    dim_rows = (2556, 3000, 20_000, 320_000)
    dims, preds, fact = star_setup(sel, ctx, 3_000_003, dim_rows)
    bitmaps_gpu, bitmaps_cpu, nbits = [], [], []
    for d, (t, p) in enumerate(zip(dims, preds)):
        dt = sel.device_table(ctx, t)
        prog = ctx.program(dt, p)
        bm = torch.full(((t.nrows + 31) // 32,), -1, dtype=torch.int32, device="cuda")
        st, cnt = ctx.pushdown_keybitmap(dt, 0, 0, prog, bm, t.nrows)
        ost, ocnt, owords = oracle.Oracle(t).keybitmap(p, 0, 0, t.nrows)
        assert st == sel.SEL_OK and ost == 0 and cnt == ocnt
        np.testing.assert_array_equal(as_u32(bm), owords)
        bitmaps_gpu.append(bm)
        bitmaps_cpu.append(owords)
        nbits.append(t.nrows)
    dfact = sel.device_table(ctx, fact)
    ofact = oracle.Oracle(fact)
    want = ofact.star_count([0, 1, 2, 3], bitmaps_cpu, nbits, threads=8)
    got = ctx.star_count(dfact, [0, 1, 2, 3], bitmaps_gpu, nbits)
    assert got == want
    fp = datagen.star_fact_predicate()
    want2 = ofact.star_count([0, 1, 2, 3], bitmaps_cpu, nbits, fp, threads=8)
    got2 = ctx.star_count(dfact, [0, 1, 2, 3], bitmaps_gpu, nbits, ctx.program(dfact, fp))
    assert got2 == want2
    # a subset of dimensions, and a single one
    assert ctx.star_count(dfact, [1, 3], [bitmaps_gpu[1], bitmaps_gpu[3]], [nbits[1], nbits[3]]) == \
        ofact.star_count([1, 3], [bitmaps_cpu[1], bitmaps_cpu[3]], [nbits[1], nbits[3]], threads=8)
    assert ctx.star_count(dfact, [0], [bitmaps_gpu[0]], [nbits[0]]) == \
        ofact.star_count([0], [bitmaps_cpu[0]], [nbits[0]], threads=8)


def test_keybitmap_edges(sel, ctx):
    t = datagen.star_dims(sizes=(100, 40, 70, 33))[1]
    dt = sel.device_table(ctx, t)
    bm = torch.zeros(8, dtype=torch.int32, device="cuda")
    # every row qualifies (no program), keys offset by key_min
    st, cnt = ctx.pushdown_keybitmap(dt, 0, -3, None, bm, 43)
    ost, ocnt, owords = oracle.Oracle(t).keybitmap(None, 0, -3, 43)
    assert (st, cnt) == (sel.SEL_OK, ocnt) and ost == 0
    np.testing.assert_array_equal(as_u32(bm)[:len(owords)], owords)
    # a qualifying key outside [key_min, key_min + nbits) is reported
    st, cnt = ctx.pushdown_keybitmap(dt, 0, 5, None, bm, 40)
    assert st == sel.SEL_E_RANGE


def test_cfg2_full_size(sel, ctx):
    """cfg2 at its full 300M rows in the default launch shape: exact count
    and the whole ascending row-id arrays (1.62M ids, and 270M ids of a 90 %
    date range) against the oracle over 16 row ranges."""
    say("cfg2 full: generating 300M rows")
    t = datagen.cfg2()
    dt = sel.device_table(ctx, t)
    tree = datagen.cfg2_predicate()
    prog = ctx.program(dt, tree)
    say("cfg2 full: GPU count")
    got = ctx.count(dt, prog)
    say("cfg2 full: oracle count")
    orc = oracle.Oracle(t)
    want = orc.count(tree, threads=16)
    assert got == want
    say(f"cfg2 full: count {got}; GPU row ids")
    out = torch.empty(got + 16, dtype=torch.int32, device="cuda")
    st, cnt = ctx.pushdown_rowids(dt, prog, UINT64_MAX, out)
    assert (st, cnt) == (sel.SEL_OK, want)
    ids = as_u32(out)[:cnt].astype(np.int64)
    say("cfg2 full: oracle row ids over 16 row ranges")
    np.testing.assert_array_equal(ids, orc.rowids(tree, threads=16).astype(np.int64))
    # the selection's projected columns (date, qty, price with NULLs, s25)
    # gathered at its ids, against numpy indexing of the host table
    cols = [0, 1, 3, 5]
    outs = [torch.empty(cnt, dtype=getattr(torch, {"i8": "int8", "i32": "int32", "i64": "int64"}[
        t.columns[c].type]), device="cuda") for c in cols]
    vouts = [torch.empty((cnt + 31) // 32, dtype=torch.int32, device="cuda") for _ in cols]
    ctx.gather(dt, out, cnt, cols, outs, vouts)
    for c, o, vo, (wv, wvalid) in zip(cols, outs, vouts, oracle.gather(t, ids, cols)):
        np.testing.assert_array_equal(o.cpu().numpy(), wv)
        bits = np.unpackbits(as_u32(vo).view(np.uint8), bitorder="little")[:cnt].astype(bool)
        np.testing.assert_array_equal(bits, wvalid)
    del out, outs, vouts
    # the sparse int64 IN lists the benchmark sweeps (10, 100 and 1000
    # values, half of them present)
    for k in (10, 100, 1000):
        tree_in = ("in", 3, datagen.sparse_in_values(t.col("price").data, k))
        prog_in = ctx.program(dt, tree_in)
        got_in = ctx.count(dt, prog_in)
        say(f"cfg2 full: IN list of {k} values, count {got_in}")
        assert got_in == orc.count(tree_in, threads=16), k
    # a date range holding about 90 % of the rows: 270M ascending ids (1.08
    # GB), the limit one below the count refuses them, the count itself
    # accepts them
    wide = ("between", 0, 0, 2300)
    prog = ctx.program(dt, wide)
    want = orc.count(wide, threads=16)
    say(f"cfg2 full: 90 % range, count {want}")
    out = torch.empty(want + 16, dtype=torch.int32, device="cuda")
    st, cnt = ctx.pushdown_rowids(dt, prog, want - 1, out)
    assert (st, cnt) == (sel.SEL_OVER_LIMIT, want)
    st, cnt = ctx.pushdown_rowids(dt, prog, want, out)
    assert (st, cnt) == (sel.SEL_OK, want)
    ids = as_u32(out)[:cnt]
    say("cfg2 full: oracle row ids of the 90 % range over 16 row ranges")
    want_ids = orc.rowids(wide, threads=16)
    np.testing.assert_array_equal(ids, want_ids)
    del dt, out, ids, want_ids
    torch.cuda.empty_cache()


def test_star_full_dimensions(sel, ctx):
    """The star probe at the star workload's own dimension sizes (2556 / 30k
    / 200k / 3.2M keys: 29 KB of bitmaps staged in LDS beside the 400 KB one
    read through the caches) over 20M fact rows: key bitmaps word for word,
    the star count with and without the fact predicate, on every subset of
    two dimensions, and star programs through sel_count and sel_count_batch,
    all against the oracle."""
    sizes = datagen.CFG4_DIM_ROWS
    assert tuple(sizes) == (2556, 30_000, 200_000, 3_200_000)
    say("star full dims: generating dimensions and 20M fact rows")
    dims, preds, fact = star_setup(sel, ctx, 20_000_003, sizes)
    bitmaps_gpu, bitmaps_cpu, nbits = [], [], []
    ddims = []
    for t, p in zip(dims, preds):
        dt = sel.device_table(ctx, t)
        ddims.append(dt)
        bm = torch.full(((t.nrows + 31) // 32,), -1, dtype=torch.int32, device="cuda")
        st, cnt = ctx.pushdown_keybitmap(dt, 0, 0, ctx.program(dt, p), bm, t.nrows)
        ost, ocnt, owords = oracle.Oracle(t).keybitmap(p, 0, 0, t.nrows)
        assert st == sel.SEL_OK and ost == 0 and cnt == ocnt
        np.testing.assert_array_equal(as_u32(bm), owords)
        bitmaps_gpu.append(bm)
        bitmaps_cpu.append(owords)
        nbits.append(t.nrows)
    dfact = sel.device_table(ctx, fact)
    ofact = oracle.Oracle(fact)
    fp = datagen.star_fact_predicate()
    fprog = ctx.program(dfact, fp)
    say("star full dims: star counts")
    every = [0, 1, 2, 3]
    want = ofact.star_count(every, bitmaps_cpu, nbits, threads=16)
    assert ctx.star_count(dfact, every, bitmaps_gpu, nbits) == want
    want_fp = ofact.star_count(every, bitmaps_cpu, nbits, fp, threads=16)
    assert ctx.star_count(dfact, every, bitmaps_gpu, nbits, fprog) == want_fp
    for a in range(4):
        for b in range(a + 1, 4):
            sub = [a, b]
            assert ctx.star_count(dfact, sub, [bitmaps_gpu[a], bitmaps_gpu[b]],
                                  [nbits[a], nbits[b]]) == \
                ofact.star_count(sub, [bitmaps_cpu[a], bitmaps_cpu[b]], [nbits[a], nbits[b]],
                                 threads=16), sub
    say("star full dims: star programs, plain and batched")
    progs = [ctx.star_program(dfact, every, bitmaps_gpu, nbits),
             ctx.star_program(dfact, every, bitmaps_gpu, nbits, fprog)]
    wants = [want, want_fp]
    keep = []
    for k, combo in enumerate(datagen.star_dim_programs(11, 6, dims)):
        bms_gpu, bms_cpu = [], []
        for d, dt, p in zip(dims, ddims, combo):
            bm = torch.empty((d.nrows + 31) // 32, dtype=torch.int32, device="cuda")
            st, _ = ctx.pushdown_keybitmap(dt, 0, 0, ctx.program(dt, p), bm, d.nrows)
            assert st == sel.SEL_OK
            ost, _, owords = oracle.Oracle(d).keybitmap(p, 0, 0, d.nrows)
            assert ost == 0
            np.testing.assert_array_equal(as_u32(bm), owords)
            bms_gpu.append(bm)
            bms_cpu.append(owords)
        keep.append(bms_gpu)
        pred = fprog if k % 2 else None
        progs.append(ctx.star_program(dfact, every, bms_gpu, nbits, pred))
        wants.append(ofact.star_count(every, bms_cpu, nbits, fp if pred is not None else None,
                                      threads=16))
    pairs = [(dfact, p) for p in progs]
    assert [ctx.count(*p) for p in pairs] == wants
    assert ctx.count_batch(pairs) == wants
    del dfact, ddims, bitmaps_gpu, keep, progs, pairs
    torch.cuda.empty_cache()
