"""The seeded generator: thread-count independence and marginal sanity."""
import numpy as np

import datagen


def test_thread_independent():
    a = datagen.lineorder_like("a", 100_003, seed=5, threads=1)
    b = datagen.lineorder_like("b", 100_003, seed=5, threads=7)
    for ca, cb in zip(a.columns, b.columns):
        assert datagen.checksum(ca.data) == datagen.checksum(cb.data), ca.name
        if ca.valid is not None:
            assert datagen.checksum(ca.valid) == datagen.checksum(cb.valid)


def test_marginals():
    n = 400_000
    t = datagen.lineorder_like("m", n, seed=11)
    d = t.col("date").data
    assert d.min() == 0 and d.max() == 2556
    # uniform: chi-square over 2557 days stays near its mean (dof 2556)
    h = np.bincount(d, minlength=2557)
    chi2 = float(((h - n / 2557) ** 2 / (n / 2557)).sum())
    assert chi2 < 2556 + 6 * np.sqrt(2 * 2556)
    q = t.col("qty").data
    assert q.min() == 1 and q.max() == 50
    # Zipf(1.1) over 25 codes: code 0 share near its probability
    s25 = t.col("s25").data
    p0 = datagen.zipf_pmf(1.1, 25)[0]
    assert abs((s25 == 0).mean() - p0) < 5 * np.sqrt(p0 * (1 - p0) / n)
    price = t.col("price")
    rate = price.null_count / n
    assert abs(rate - 0.05) < 5 * np.sqrt(0.05 * 0.95 / n)
    valid = np.unpackbits(price.valid.view(np.uint8), bitorder="little")[:n].astype(bool)
    assert int((~valid).sum()) == price.null_count
    assert np.all(price.data[~valid] == datagen.CFG2_PRICE_NULL_FILL)
    # log-normal(10, 1): median near e^10
    med = float(np.median(price.data[valid]))
    assert abs(np.log(med) - 10.0) < 0.02


def test_seed_changes_stream():
    a = datagen.uniform("i32", 1, 0, 0, 9999, 1000)
    b = datagen.uniform("i32", 2, 0, 0, 9999, 1000)
    c = datagen.uniform("i32", 1, 1, 0, 9999, 1000)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_cfg3_programs_shape():
    progs = datagen.cfg3_programs()
    assert len(progs) == 64
    assert [t for t, _ in progs] == [k // 16 for k in range(64)]
    leaves = [datagen.tree_leaves(tree) for _, tree in progs]
    assert min(leaves) >= 2 and max(leaves) <= 8
    # same seed, same programs
    again = datagen.cfg3_programs()
    assert repr(again[:5]) == repr(progs[:5])


def test_serving_trace_shape():
    tr = datagen.serving_trace(seed=52, rate=2000.0, duration=2.0)
    n = len(tr)
    assert abs(n - 4000) < 5 * np.sqrt(4000)                 # Poisson count
    assert all(a < b for a, b in zip([t for t, _, _ in tr], [t for t, _, _ in tr][1:]))
    ks = [len(items) for _, items, _ in tr]
    assert min(ks) == 1 and max(ks) == 12
    frac = sum(1 for *_, pd in tr if pd) / n
    assert abs(frac - 0.1) < 0.03
    assert all(pd[0] != 4 for *_, pd in tr if pd)             # no push-down on the star table
