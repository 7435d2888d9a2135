"""GPU: projected columns of a materialised selection (sel_gather through the
C ABI) against the oracle's gather, bit-exact on every value and every
validity bit."""
import numpy as np
import pytest

import datagen
import oracle
from tests import sqlite_ref
from tests.gpu_common import UINT64_MAX, as_u32, ids_tensor, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TORCH_DT = {"i8": "int8", "i16": "int16", "i32": "int32", "i64": "int64"}


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


def valid_words(valid: np.ndarray) -> np.ndarray:
    bits = np.packbits(valid.astype(np.uint8), bitorder="little")
    buf = np.zeros((valid.size + 31) // 32 * 4, dtype=np.uint8)
    buf[: bits.size] = bits
    return buf.view(np.uint32)


def gather_and_check(sel, ctx, t, dt, ids_dev, ids_host, cols):
    count = ids_host.size
    outs = [torch.full((max(1, count),), 77, dtype=getattr(torch, TORCH_DT[t.columns[c].type]),
                       device="cuda") for c in cols]
    vouts = [torch.full((max(1, (count + 31) // 32),), -1, dtype=torch.int32, device="cuda")
             for _ in cols]
    ctx.gather(dt, ids_dev, count, cols, outs, vouts)
    want = oracle.gather(t, ids_host, cols)
    for (wv, wvalid), o, vo in zip(want, outs, vouts):
        np.testing.assert_array_equal(o.cpu().numpy()[:count], wv)
        nw = (count + 31) // 32
        np.testing.assert_array_equal(as_u32(vo)[:nw], valid_words(wvalid)[:nw])


@pytest.mark.parametrize("n", [1, 65, 2049, 100_003])
def test_gather_selected_rows(sel, ctx, n):
    """Random programs over a random table of every type with NULLs: the ids
    of each selection, then every column gathered at them."""
    say(f"gather n={n}")
    rng = np.random.default_rng(80_000 + n)
    t = datagen.random_table(rng, n, grid=False, null_rate=0.3)
    dt = sel.device_table(ctx, t)
    cols = list(range(len(t.columns)))
    for _ in range(4):
        tree = sqlite_ref.clamp_literals(datagen.random_tree(rng, t, grid=False))
        prog = ctx.program(dt, tree)
        want_ids = oracle.Oracle(t).rowids(tree)
        out = ids_tensor(want_ids.size, torch)
        st, cnt = ctx.pushdown_rowids(dt, prog, UINT64_MAX, out)
        assert st == sel.SEL_OK and cnt == want_ids.size
        gather_and_check(sel, ctx, t, dt, out, want_ids, cols)


def test_gather_any_order_and_edges(sel, ctx):
    """Ids in any order (a permutation, repeats, the last row), counts that
    end inside a validity word, no ids at all, and ids past the table, which
    are an error."""
    rng = np.random.default_rng(81_000)
    n = 50_021
    t = datagen.random_table(rng, n, grid=False, null_rate=0.2)
    dt = sel.device_table(ctx, t)
    cols = [3, 0, 2, 1, 3]
    for count in (1, 31, 32, 33, 63, 64, 65, 1000, n):
        ids = rng.permutation(n)[:count].astype(np.uint32)
        ids[0] = n - 1
        if count > 2:
            ids[1] = ids[2]
        dev = torch.from_numpy(ids.view(np.int32)).cuda()
        gather_and_check(sel, ctx, t, dt, dev, ids, cols)
    outs = [torch.empty(1, dtype=torch.int8, device="cuda")]
    ctx.gather(dt, None, 0, [0], outs)
    bad = torch.tensor([5, n, 7], dtype=torch.int32, device="cuda")
    outs = [torch.empty(3, dtype=getattr(torch, TORCH_DT[t.columns[0].type]), device="cuda")]
    with pytest.raises(sel.SelError):
        ctx.gather(dt, bad, 3, [0], outs)
    with pytest.raises(sel.SelError):
        ctx.gather(dt, bad, 3, [len(t.columns)], outs)
