"""Pins of the CPU oracle against things other than itself.

Each check returns a list of failure strings (empty = pass) so that the
same battery can be run against deliberately broken builds of the oracle
(tests/test_oracle_mutants.py) to show that it catches plausible mistakes.

Pins used:
  * Kleene / SQL truth tables from tests/golden/kleene_k3.txt
  * SQLite (an independent SQL engine) on small random tables with NULLs
  * closed forms on constructed columns (permutations, NULL counts,
    numpy.bincount for code sets)
  * invariants of three-valued logic and of Algorithm 1's limit check
  * brute-force nested-loop star joins in SQLite
"""
from __future__ import annotations

import os

import numpy as np

import datagen
import oracle
from tests import sqlite_ref

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
SYM = {"T": oracle.T, "U": oracle.U, "F": oracle.F}


def _leaf_table(values):
    """One int32 column x0 with the given values; None = NULL."""
    n = len(values)
    data = np.array([0 if v is None else v for v in values], dtype=np.int32)
    words = np.zeros((n + 31) // 32, dtype=np.uint32)
    for i, v in enumerate(values):
        if v is not None:
            words[i // 32] |= np.uint32(1 << (i % 32))
    t = datagen.Table("leaf", n)
    t.columns.append(datagen.Column("x0", "i32", data, words))
    t.columns.append(datagen.Column("x1", "i32", data.copy(), words.copy()))
    return t


def check_kleene(lib_path=None):
    """Leaf ('cmp', c, '=', 1) is T on 1, F on 0, U on NULL; combine two such
    leaves over all 9 (a, b) rows and compare with the golden tables."""
    fails = []
    vals = {"T": 1, "F": 0, "U": None}
    rows = []
    with open(os.path.join(GOLDEN, "kleene_k3.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                rows.append(line)
    for op, a, b, res in rows:
        if b == "-":
            t = _leaf_table([vals[a]])
            leaf = ("cmp", 0, "=", 1)
            tree = ("not", leaf) if op == "NOT" else ("isunknown", leaf)
        else:
            t = _leaf_table([vals[a]])
            t.columns[1].data[:] = 0 if vals[b] is None else vals[b]
            t.columns[1].valid[:] = 0 if vals[b] is None else 1
            tree = (op.lower(), ("cmp", 0, "=", 1), ("cmp", 1, "=", 1))
        got = oracle.Oracle(t, lib_path).eval_row(tree, 0)
        if got != SYM[res]:
            fails.append(f"kleene {op} {a} {b}: got {got} want {res}")
    return fails


def check_sqlite(lib_path=None, seeds=range(12), n=400):
    """Random predicates over random tables: counts, row ids and per-row
    truth values equal SQLite's."""
    fails = []
    for s in seeds:
        rng = np.random.default_rng(1000 + s)
        t = datagen.random_table(rng, n, grid=(s % 2 == 0), null_rate=0.25)
        db = sqlite_ref.connect(t)
        o = oracle.Oracle(t, lib_path)
        for _ in range(12):
            tree = sqlite_ref.clamp_literals(datagen.random_tree(rng, t, grid=(s % 2 == 0)))
            want = sqlite_ref.truth(db, tree)
            got = o.eval_all(tree)
            if not np.array_equal(want, got):
                fails.append(f"sqlite truth seed {s}: {tree!r:.200}")
                continue
            c = o.count(tree)
            if c != int((want == 2).sum()) or c != sqlite_ref.count(db, tree):
                fails.append(f"sqlite count seed {s}")
            ids = o.rowids(tree)
            want_ids = sqlite_ref.rowids(db, tree)
            if not np.array_equal(ids, want_ids):
                fails.append(f"sqlite rowids seed {s}")
            # the row-range split: ranges of 28-29 rows, most holding some ids
            if not np.array_equal(o.rowids(tree, threads=7), want_ids):
                fails.append(f"sqlite rowids over 7 row ranges seed {s}")
    return fails


def check_closed_forms(lib_path=None, n=20000):
    fails = []
    rng = np.random.default_rng(7)
    perm = rng.permutation(n).astype(np.int32)
    t = datagen.Table("perm", n)
    t.columns.append(datagen.Column("p", "i32", perm))
    # a narrow-type permutation-like column: every int8 value equally often
    t.columns.append(datagen.Column("b", "i8", (np.arange(n) % 256 - 128).astype(np.int8)))
    o = oracle.Oracle(t, lib_path)
    cases = []
    for _ in range(8):
        a, b = sorted(int(x) for x in rng.integers(0, n, 2))
        cases.append((("between", 0, a, b), b - a + 1))
        v = int(rng.integers(0, n))
        cases += [(("cmp", 0, "<", v), v), (("cmp", 0, "<=", v), v + 1),
                  (("cmp", 0, ">", v), n - v - 1), (("cmp", 0, ">=", v), n - v),
                  (("cmp", 0, "=", v), 1), (("cmp", 0, "<>", v), n - 1)]
        k = int(rng.integers(1, 20))
        vals = [int(x) for x in rng.choice(n, k, replace=False)]
        cases.append((("in", 0, tuple(vals + vals[:2])), k))   # duplicates count once
    cases += [(("between", 0, 10, 5), 0), (("cmp", 0, ">=", -(2 ** 63)), n),
              (("in", 0, (-1, n)), 0), (("true",), n), (("false",), 0)]
    per = n // 256
    rem = n % 256
    # int8 column: value v appears per (+1 if its position < rem) times
    cnt8 = lambda v: per + (1 if (v + 128) < rem else 0)
    cases += [(("cmp", 1, "<", 0), sum(cnt8(v) for v in range(-128, 0))),
              (("cmp", 1, "=", -128), cnt8(-128)), (("cmp", 1, ">", 126), cnt8(127)),
              (("between", 1, -1, 1), cnt8(-1) + cnt8(0) + cnt8(1))]
    for tree, want in cases:
        got = o.count(tree)
        if got != want:
            fails.append(f"closed form {tree!r:.120}: got {got} want {want}")
    ids = o.rowids(("between", 0, 100, 199))
    if not np.array_equal(np.sort(perm[ids]), np.arange(100, 200, dtype=np.int32)):
        fails.append("closed form: ids of a permutation range")

    # NULL counts: generator's own record and numpy's popcount of validity
    t2 = datagen.lineorder_like("nulls", 50_000, seed=9)
    o2 = oracle.Oracle(t2, lib_path)
    price = t2.col("price")
    pop = int(np.unpackbits(price.valid.view(np.uint8), bitorder="little")[: t2.nrows].sum())
    if o2.count(("isnull", 3)) != price.null_count or o2.count(("notnull", 3)) != pop:
        fails.append("closed form: IS NULL / IS NOT NULL counts")
    # code sets: sum of numpy.bincount over the set codes
    words = datagen.cfg2_like_bitmap()
    codes = sqlite_ref.codes_of(words, 4500)
    hist = np.bincount(t2.col("s4500").data, minlength=4500)
    if o2.count(("codeset", 6, 4500, words)) != int(hist[codes].sum()):
        fails.append("closed form: CODESET = bincount dot bitmap")
    # a tautology and a contradiction over a nullable predicate
    p = ("cmp", 3, ">=", 20000)
    if o2.count(("or", p, ("not", p), ("isunknown", p))) != t2.nrows:
        fails.append("closed form: p OR NOT p OR p IS UNKNOWN = N")
    if o2.count(("and", p, ("not", p))) != 0:
        fails.append("closed form: p AND NOT p = 0")
    return fails


def check_invariants(lib_path=None, n=30000, seeds=range(4)):
    fails = []
    for s in seeds:
        rng = np.random.default_rng(500 + s)
        t = datagen.random_table(rng, n, grid=False, null_rate=0.2)
        o = oracle.Oracle(t, lib_path)
        for _ in range(6):
            p = datagen.random_tree(rng, t, max_depth=4, max_leaves=6, grid=False)
            q = datagen.random_tree(rng, t, max_depth=4, max_leaves=6, grid=False)
            cp, cnp, cup = o.count(p), o.count(("not", p)), o.count(("isunknown", p))
            if cp + cnp + cup != n:
                fails.append(f"invariant T+F+U=N seed {s}")
            cpq, cpnq = o.count(("and", p, q)), o.count(("and", p, ("not", q)))
            vp, vq = o.eval_all(p), o.eval_all(q)
            tu = int(((vp == 2) & (vq == 1)).sum())
            if cpq + cpnq + tu != cp:
                fails.append(f"invariant p AND q + p AND NOT q seed {s}")
            if not 0 <= cp <= n:
                fails.append("selectivity outside [0,1]")
            if o.count(("or", p, q)) != cp + o.count(q) - cpq:
                fails.append(f"inclusion-exclusion seed {s}")
            if o.count(("not", ("and", p, q))) != o.count(("or", ("not", p), ("not", q))):
                fails.append(f"De Morgan seed {s}")
            if o.count(("and", q, p)) != cpq or o.count(("or", q, p)) != o.count(("or", p, q)):
                fails.append(f"commutativity seed {s}")
            ids = o.rowids(p)
            if ids.size != cp or (ids.size > 1 and not np.all(np.diff(ids.astype(np.int64)) > 0)):
                fails.append(f"row ids ascending, len = count, seed {s}")
            if o.count(p, threads=5) != cp:
                fails.append(f"threaded count seed {s}")
            if not np.array_equal(o.rowids(p, threads=5), ids):
                fails.append(f"threaded row ids seed {s}")
    return fails


def check_limits(lib_path=None):
    """Algorithm 1: count > maxSize aborts; count == maxSize materialises."""
    fails = []
    t = datagen.cfg1(20000, seed=3)
    o = oracle.Oracle(t, lib_path)
    p = datagen.cfg1_predicate()
    c = o.count(p)
    ids = o.rowids(p)
    st, cnt, got = o.pushdown(p, c - 1, t.nrows)
    if (st, cnt, got) != (1, c, None):
        fails.append("limit: count-1 must abort")
    st, cnt, got = o.pushdown(p, c, t.nrows)
    if st != 0 or cnt != c or not np.array_equal(got, ids):
        fails.append("limit: count == max_rows materialises")
    st, cnt, got = o.pushdown(p, 2 ** 64 - 1, c - 1)
    if st != 2 or cnt != c:
        fails.append("limit: capacity")
    st, cnt, got = o.pushdown(("false",), 0, 10)
    if st != 0 or cnt != 0:
        fails.append("limit: an empty result is accepted with max_rows = 0")
    return fails


def check_star(lib_path=None, seeds=range(3)):
    """Star semi-join count == SQLite join count; key bitmaps == numpy."""
    fails = []
    for s in seeds:
        rng = np.random.default_rng(900 + s)
        sizes = (int(rng.integers(5, 40)), int(rng.integers(5, 60)))
        dims = []
        for d, rows in enumerate(sizes):
            t = datagen.Table(f"d{d}", rows)
            key_min = int(rng.integers(-3, 4))
            t.columns.append(datagen.Column("key", "i32",
                                            (np.arange(rows) + key_min).astype(np.int32)))
            t.columns.append(datagen.Column("a", "i32", rng.integers(0, 5, rows).astype(np.int32)))
            dims.append((t, key_min))
        nf = 600
        fact = datagen.Table("f", nf)
        for d, rows in enumerate(sizes):
            # foreign keys mostly valid, some dangling (-1, rows+2)
            fk = rng.integers(-1, rows + 2, nf).astype(np.int32)
            fact.columns.append(datagen.Column(f"fk{d}", "i32", fk))
        fact.columns.append(datagen.Column("m", "i32", rng.integers(0, 10, nf).astype(np.int32)))
        preds = [("cmp", 1, "<", int(rng.integers(1, 5))), ("in", 1, (0, 3))]
        bitmaps, nbits = [], []
        for (t, key_min), p in zip(dims, preds):
            o = oracle.Oracle(t, lib_path)
            st, cnt, words = o.keybitmap(p, 0, key_min, t.nrows)
            mask = o.eval_all(p) == 2
            want = np.zeros_like(words)
            for k in (t.columns[0].data[mask].astype(np.int64) - key_min):
                want[k // 32] |= np.uint32(1 << (k % 32))
            if st != 0 or cnt != int(mask.sum()) or not np.array_equal(words, want):
                fails.append(f"keybitmap seed {s}")
            bitmaps.append(words)
            nbits.append(t.nrows)
            # keys are bitmap positions: fact fk values index bits directly
        fo = oracle.Oracle(fact, lib_path)
        fpred = ("cmp", 2, ">=", 4)
        for pred in (None, fpred):
            got = fo.star_count([0, 1], bitmaps, nbits, pred)
            # the same count with the fact rows split into ranges over threads
            split = [fo.star_count([0, 1], bitmaps, nbits, pred, threads=k) for k in (5, 16)]
            import sqlite3
            db = sqlite3.connect(":memory:")
            db.execute("CREATE TABLE f (fk0 INTEGER, fk1 INTEGER, m INTEGER)")
            db.executemany("INSERT INTO f VALUES (?,?,?)",
                           [tuple(int(c.data[i]) for c in fact.columns) for i in range(nf)])
            for d, ((t, key_min), p) in enumerate(zip(dims, preds)):
                db.execute(f"CREATE TABLE d{d} (pos INTEGER, a INTEGER)")
                # the bitmap is indexed by key - key_min: join on that position
                db.executemany(f"INSERT INTO d{d} VALUES (?,?)",
                               [(int(t.columns[0].data[i]) - key_min, int(t.columns[1].data[i]))
                                for i in range(t.nrows)])
            w = [sqlite_ref.to_sql(p).replace("x1", f"d{d}.a") for d, p in enumerate(preds)]
            if pred is not None:
                w.append("f.m >= 4")
            sql = ("SELECT COUNT(*) FROM f JOIN d0 ON f.fk0 = d0.pos JOIN d1 ON f.fk1 = d1.pos "
                   f"WHERE {' AND '.join(w)}")
            want = int(db.execute(sql).fetchone()[0])
            if got != want:
                fails.append(f"star count seed {s} pred {pred}: got {got} want {want}")
            for k, c in zip((5, 16), split):
                if c != want:
                    fails.append(f"star count over {k} row ranges seed {s} pred {pred}: got {c} want {want}")
            # bits past nbits in the last word are outside the set
            padded = [b.copy() for b in bitmaps]
            for b, nb in zip(padded, nbits):
                if nb % 32:
                    b[-1] |= np.uint32((0xFFFFFFFF << (nb % 32)) & 0xFFFFFFFF)
            if fo.star_count([0, 1], padded, nbits, pred) != want:
                fails.append(f"star count seed {s}: bits beyond nbits matched")
        # a qualifying key outside the bitmap range is reported
        t, key_min = dims[0]
        st, _, _ = oracle.Oracle(t, lib_path).keybitmap(None, 0, key_min + 1, t.nrows)
        if st != -6:
            fails.append("keybitmap: out-of-range key not reported")
    return fails


ALL = [check_kleene, check_sqlite, check_closed_forms, check_invariants, check_limits, check_star]


def battery(lib_path=None, quick=False):
    fails = []
    for chk in ALL:
        if quick and chk is check_sqlite:
            fails += chk(lib_path, seeds=range(4), n=200)
        elif quick and chk is check_invariants:
            fails += chk(lib_path, n=5000, seeds=range(2))
        else:
            fails += chk(lib_path)
    return fails
