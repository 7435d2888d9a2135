"""The row-id push-down that allocates nothing (sel_pushdown_rowids_noalloc,
for callers that cannot allocate device memory) against the allocating
sel_pushdown_rowids and the oracle, through the C ABI: statuses, counts and
whole id arrays bit-exact on two calls in a row, the second on a smaller
table, and the size limit of its fixed workspace."""
import numpy as np
import pytest

import datagen
import oracle
from tests.gpu_common import UINT64_MAX, as_u32, ids_tensor, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SENTINEL = 0xDEADBEEF


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


def both(sel, ctx, dt, prog, max_rows, n_out, cap=None):
    """(status, count, ids buffer) of the plain call and of the call that
    allocates nothing, each into its own sentinel-filled buffer."""
    res = []
    for call in (ctx.pushdown_rowids, ctx.pushdown_rowids_noalloc):
        out = ids_tensor(n_out, torch, SENTINEL)
        st, cnt = call(dt, prog, max_rows, out, cap)
        res.append((st, cnt, as_u32(out)))
    return res


def check_same(sel, ctx, dt, orc, tree, label):
    """Unlimited push-down, then the limit forced to count-1 and the
    capacity to count-1: the two entry points agree everywhere, and the ids
    equal the oracle's."""
    prog = ctx.program(dt, tree)
    want = orc.count(tree, threads=8)
    want_ids = orc.rowids(tree, threads=8)
    say(f"no-alloc push-down: {label}, {dt.nrows} rows, {want} TRUE")
    (s0, c0, o0), (s1, c1, o1) = both(sel, ctx, dt, prog, UINT64_MAX, want + 5)
    assert (s0, c0) == (s1, c1) == (sel.SEL_OK, want)
    np.testing.assert_array_equal(o1, o0)
    np.testing.assert_array_equal(o1[:want], want_ids)
    assert np.all(o1[want:] == SENTINEL)
    if want > 0:
        (s0, c0, o0), (s1, c1, o1) = both(sel, ctx, dt, prog, want - 1, want + 5)
        assert (s0, c0) == (s1, c1) == (sel.SEL_OVER_LIMIT, want)
        assert np.all(o1 == SENTINEL) and np.all(o0 == SENTINEL)
        (s0, c0, o0), (s1, c1, o1) = both(sel, ctx, dt, prog, UINT64_MAX, want + 5, cap=want - 1)
        assert (s0, c0) == (s1, c1) == (sel.SEL_E_CAPACITY, want)
        assert np.all(o1 == SENTINEL) and np.all(o0 == SENTINEL)
    return want


def test_two_calls_second_smaller(sel, ctx):
    """A 6-leaf selection over 3 000 017 rows (1466 tiles, ragged tail),
    then 100 003 rows of another table: the second call runs on whatever
    the first left in the shared workspace."""
    big = datagen.cfg2(n=3_000_017, seed=71)
    dt_big = sel.device_table(ctx, big)
    c_big = check_same(sel, ctx, dt_big, oracle.Oracle(big), datagen.cfg2_predicate(0, 1500), "cfg2-like")
    assert c_big > 10_000
    small = datagen.cfg1(100_003, seed=72)
    dt_small = sel.device_table(ctx, small)
    c_small = check_same(sel, ctx, dt_small, oracle.Oracle(small), datagen.cfg1_predicate(), "3 x int32")
    assert 0 < c_small < c_big


@pytest.mark.parametrize("n", [0, 1, 2047, 2049])
def test_tiny_and_empty(sel, ctx, n):
    t = datagen.cfg1(n, seed=73)
    dt = sel.device_table(ctx, t)
    check_same(sel, ctx, dt, oracle.Oracle(t), ("cmp", 0, "<", 5000), f"n={n}")


def test_dense_selection_after_sparse(sel, ctx):
    """Every mask word written (a 90 % range) right after a sparse call."""
    t = datagen.cfg2(n=2_000_000, seed=74)
    dt = sel.device_table(ctx, t)
    orc = oracle.Oracle(t)
    check_same(sel, ctx, dt, orc, ("between", 0, 0, 2300), "90 % date range")
    check_same(sel, ctx, dt, orc, datagen.cfg2_predicate(365, 729), "6 leaves")


def test_table_beyond_fixed_workspace(sel, ctx):
    """A table whose workspace exceeds the fixed 64 MiB is refused before
    any launch; the allocating call still serves it."""
    n = 600_000_000
    col = torch.zeros(n, dtype=torch.int8, device="cuda")
    col[7] = 1
    dt = ctx.table(n, [("i8", 0, col.data_ptr(), None)], keep=(col,))
    prog = ctx.program(dt, ("cmp", 0, "=", 1))
    out = ids_tensor(4, torch, SENTINEL)
    with pytest.raises(sel.SelError) as e:
        ctx.pushdown_rowids_noalloc(dt, prog, UINT64_MAX, out)
    assert e.value.status == sel.SEL_E_INVALID
    assert "workspace" in str(e.value)
    assert np.all(as_u32(out) == SENTINEL)
    assert ctx.pushdown_rowids(dt, prog, UINT64_MAX, out) == (sel.SEL_OK, 1)
    assert as_u32(out)[0] == 7
