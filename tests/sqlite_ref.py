"""SQLite as an independent reference for SQL WHERE semantics.

SQLite (the engine built into Python) implements SQL's three-valued logic,
IN-lists, BETWEEN and IS NULL on 64-bit integers.  Loading a small table
into it and asking for COUNT(*) / the qualifying rowids pins the oracle to
a textbook SQL implementation rather than to itself.
"""
from __future__ import annotations

import sqlite3

import numpy as np

INT64_MIN, INT64_MAX = -(2 ** 63), 2 ** 63 - 1


def _valid_mask(col, n):
    if col.valid is None:
        return np.ones(n, dtype=bool)
    bits = np.unpackbits(col.valid.view(np.uint8), bitorder="little")[:n]
    return bits.astype(bool)


def connect(table):
    """In-memory SQLite table r(rid, x0, x1, ...) with NULLs."""
    db = sqlite3.connect(":memory:")
    names = [f"x{k}" for k in range(len(table.columns))]
    db.execute(f"CREATE TABLE r (rid INTEGER PRIMARY KEY, {', '.join(n + ' INTEGER' for n in names)})")
    cols = []
    for c in table.columns:
        v = _valid_mask(c, table.nrows)
        cols.append([int(x) if ok else None for x, ok in zip(c.data.tolist(), v.tolist())])
    rows = [(i, *[cols[k][i] for k in range(len(cols))]) for i in range(table.nrows)]
    db.executemany(f"INSERT INTO r VALUES ({', '.join('?' * (len(names) + 1))})", rows)
    return db


def codes_of(words, nbits):
    w = np.asarray(words, dtype=np.uint32)
    bits = np.unpackbits(w.view(np.uint8), bitorder="little")[:nbits]
    return [int(c) for c in np.flatnonzero(bits)]


def to_sql(tree) -> str:
    op = tree[0]
    if op == "true":
        return "(1=1)"
    if op == "false":
        return "(1=0)"
    if op == "cmp":
        _, k, cmp, v = tree
        return f"(x{k} {cmp} {int(v)})"
    if op == "between":
        _, k, lo, hi = tree
        return f"(x{k} BETWEEN {int(lo)} AND {int(hi)})"
    if op == "in":
        _, k, vals = tree
        return f"(x{k} IN ({', '.join(str(int(v)) for v in vals)}))"
    if op == "codeset":
        _, k, nbits, words = tree
        codes = codes_of(words, nbits)
        if not codes:
            # an empty set: FALSE for non-NULL, UNKNOWN for NULL
            return f"(x{k} <> x{k})"
        return f"(x{k} IN ({', '.join(map(str, codes))}))"
    if op == "isnull":
        return f"(x{tree[1]} IS NULL)"
    if op == "notnull":
        return f"(x{tree[1]} IS NOT NULL)"
    if op == "and":
        return "(" + " AND ".join(to_sql(k) for k in tree[1:]) + ")"
    if op == "or":
        return "(" + " OR ".join(to_sql(k) for k in tree[1:]) + ")"
    if op == "not":
        return f"(NOT {to_sql(tree[1])})"
    if op == "isunknown":
        return f"(({to_sql(tree[1])}) IS NULL)"
    raise ValueError(op)


def clamp_literals(tree):
    """Clamp literals into int64 (SQLite would round wider ones to REAL)."""
    op = tree[0]
    c = lambda v: max(INT64_MIN, min(INT64_MAX, int(v)))
    if op == "cmp":
        return ("cmp", tree[1], tree[2], c(tree[3]))
    if op == "between":
        return ("between", tree[1], c(tree[2]), c(tree[3]))
    if op == "in":
        return ("in", tree[1], tuple(c(v) for v in tree[2]))
    if op in ("and", "or", "not", "isunknown"):
        return (op, *[clamp_literals(k) for k in tree[1:]])
    return tree


def count(db, tree) -> int:
    return int(db.execute(f"SELECT COUNT(*) FROM r WHERE {to_sql(tree)}").fetchone()[0])


def rowids(db, tree) -> np.ndarray:
    rows = db.execute(f"SELECT rid FROM r WHERE {to_sql(tree)} ORDER BY rid").fetchall()
    return np.asarray([r[0] for r in rows], dtype=np.uint32)


def truth(db, tree) -> np.ndarray:
    """0 = FALSE, 1 = UNKNOWN, 2 = TRUE per row, as SQLite evaluates it."""
    rows = db.execute(f"SELECT {to_sql(tree)} FROM r ORDER BY rid").fetchall()
    out = np.empty(len(rows), dtype=np.uint8)
    for i, (v,) in enumerate(rows):
        out[i] = 1 if v is None else (2 if v else 0)
    return out
