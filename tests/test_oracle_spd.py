"""CPU pins of the oracle's Algorithm 1 (EvaluateAndPushDown, Ch.4 sec.4.2)
and of its projected-column gather (Ch.3 sec.3.3).

The relations here have a column that holds the row index, so a range
predicate [a, b] selects exactly rows a..b: every count and id list below is
written out by hand from that closed form, and every queue decision from the
algorithm's text (threshold with strict >, largest relation popped, then the
others by descending size, each pushed iff count <= maxSize)."""
import numpy as np
import pytest

import datagen
import oracle


def rel(n, name="r"):
    t = datagen.Table(name, n)
    t.columns.append(datagen.Column("id", "i32", np.arange(n, dtype=np.int32)))
    return t


def rng_(a, b):
    return ("between", 0, a, b)


def test_queue_threshold_probe_and_order():
    A, B, C, D, E, F = rel(5000), rel(200), rel(80000), rel(3000), rel(3000), rel(1000)
    r = oracle.select_pushdown(
        [(A, rng_(0, 249)), (B, rng_(0, 9)), (C, rng_(0, 5)), (D, rng_(10, 159)),
         (E, rng_(0, 150)), (F, rng_(0, 0))],
        min_table_size=1000, max_selectivity=0.05)
    # 200 and 1000 rows are not above the threshold; 80000 is the probe
    assert [x["decision"] for x in r] == ["pushed", "small", "probe", "pushed", "reverted", "small"]
    # the queue after the probe: 5000, then the two 3000-row relations in
    # input order
    assert [x["order"] for x in r] == [0, None, None, 1, 2, None]
    # maxSize = size * 0.05: 250, 150, 150; counts 250, 150, 151
    assert [x["max_rows"] for x in r] == [250, 10, 4000, 150, 150, 50]
    assert [x["count"] for x in r] == [250, 0, 0, 150, 151, 0]
    assert [x["status"] for x in r] == [0, 0, 0, 0, 1, 0]
    np.testing.assert_array_equal(r[0]["ids"], np.arange(0, 250))
    np.testing.assert_array_equal(r[3]["ids"], np.arange(10, 160))
    assert r[4]["ids"] is None and r[2]["ids"] is None


@pytest.mark.parametrize("c", [1, 37, 4096])
def test_limit_on_either_side(c):
    # 8192 rows and ratios j / 8192: maxSize is exactly j
    P, R = rel(100_000), rel(8192)
    out = []
    for j in (c - 1, c, c + 1):
        r = oracle.select_pushdown([(P, None), (R, rng_(100, 100 + c - 1))],
                                   max_selectivity=j / 8192)
        assert r[0]["decision"] == "probe" and r[1]["max_rows"] == j and r[1]["count"] == c
        out.append(r[1]["decision"])
    assert out == ["reverted", "pushed", "pushed"]


def test_zero_limit_and_empty_selection():
    # a zero limit still accepts an empty selection (count > maxSize is strict)
    P, R = rel(10_000), rel(5000)
    r = oracle.select_pushdown([(P, None), (R, rng_(6000, 7000))], max_selectivity=0.0)
    assert (r[1]["decision"], r[1]["count"], r[1]["max_rows"]) == ("pushed", 0, 0)
    assert r[1]["ids"].size == 0
    r = oracle.select_pushdown([(P, None), (R, rng_(4999, 7000))], max_selectivity=0.0)
    assert (r[1]["decision"], r[1]["count"]) == ("reverted", 1)


def test_full_ratio_pushes_everything_and_capacity_reverts():
    P, R, S = rel(50_000), rel(4000), rel(3000)
    r = oracle.select_pushdown([(P, rng_(0, 10)), (R, rng_(0, 3999)), (S, rng_(5, 2004), 1999)],
                               max_selectivity=1.0)
    assert [x["decision"] for x in r] == ["probe", "pushed", "reverted"]
    assert r[1]["count"] == 4000 and r[1]["max_rows"] == 4000
    np.testing.assert_array_equal(r[1]["ids"], np.arange(4000))
    # 2000 ids do not fit a buffer of 1999: reverted, count still known
    assert (r[2]["status"], r[2]["count"]) == (2, 2000)


def test_degenerate_queues():
    small = [(rel(10), rng_(0, 1)), (rel(1000), rng_(0, 1))]
    assert [x["decision"] for x in oracle.select_pushdown(small)] == ["small", "small"]
    one = oracle.select_pushdown([(rel(1001), rng_(0, 1))])
    assert one[0]["decision"] == "probe" and one[0]["count"] == 0
    # a relation without a selection can be the probe, or sit in the queue
    r = oracle.select_pushdown([(rel(3000), None), (rel(2000), None), (rel(2500), rng_(0, 9))])
    assert [x["decision"] for x in r] == ["probe", "no_pred", "pushed"]
    assert [x["order"] for x in r] == [None, 1, 0]


def test_max_size_rounding_reading():
    # the product is taken in double: 0.05 * 3 is 0.15000000000000002
    assert oracle.max_size(3, 0.05) == 0
    assert oracle.max_size(20, 0.05) == 1
    assert oracle.max_size(7, float("nan")) == 0
    assert oracle.max_size(7, -1.0) == 0 and oracle.max_size(7, 2.0) == 7
    assert oracle.max_size(300_000_000, 0.05) == 15_000_000


def test_gather_closed_forms():
    """The oracle's projected columns on columns whose value and validity are
    closed forms of the row: value 3r + 7 (wrapped to the type) and NULL
    exactly where r % 3 == 0."""
    n = 10_000
    r = np.arange(n, dtype=np.int64)
    t = datagen.Table("g", n)
    isnull = r % 3 == 0
    bits = np.packbits(~isnull, bitorder="little")
    words = np.zeros((n + 31) // 32 * 4, dtype=np.uint8)
    words[: bits.size] = bits
    words = words.view(np.uint32)
    for ty, dt in (("i8", np.int8), ("i16", np.int16), ("i32", np.int32), ("i64", np.int64)):
        t.columns.append(datagen.Column(ty, ty, (3 * r + 7).astype(dt), valid=words))
    ids = np.array([0, 1, 2, 3, 85, 86, 9_999], dtype=np.uint32)
    got = oracle.gather(t, ids, [0, 1, 2, 3])
    for (vals, valid), dt in zip(got, (np.int8, np.int16, np.int32, np.int64)):
        want = [(3 * int(i) + 7) for i in ids]
        assert [int(v) for v in vals] == [int(np.array(w).astype(dt)) for w in want]
        assert list(valid) == [int(i) % 3 != 0 for i in ids]
    # the int8 column wraps: row 85 holds 262 mod 256 = 6, row 86 holds 265 - 256 = 9
    assert int(got[0][0][4]) == 6 and int(got[0][0][5]) == 9
