"""Python front of the CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  It shares no
code with the HIP path: predicate trees (see ``datagen``) are walked
directly by the C oracle, whereas the product lowers them to a postfix
program of its own.

Every function here restates the thesis' definitions (Shin 2018):
  count     -- Ch.3 sec.3.1: exact cardinality of sigma(R) by COUNT(*)
  pushdown  -- Algorithm 1, Execute(node, isSPD, maxSize): count, abort if
               count > maxSize, else materialise sigma(R) (ascending ids)
  keybitmap -- Ch.3 sec.3.3 / Algorithm 1: a pushed-down non-probe relation,
               kept as the set of its qualifying keys
  star_count-- fact rows whose foreign keys all hit those key sets
  gather    -- Ch.3 sec.3.3: the materialised sigma(R) carries the columns
               the query projects, read at its row ids
  join_size, star_plan_cost, best_star_plan -- Ch.1 sec.1.1: the join-size
               formula and the cheapest left-deep order of a star query
  factor_counts, independence_estimate, q_error -- Ch.1 sec.1.1: the
               counts of a selection's conjuncts, the product estimate that
               assumes them independent, and its error against the count
  select_pushdown -- Algorithm 1, EvaluateAndPushDown: the size-ordered
               queue of a query's relations, the probe relation skipped, and
               Execute(compound, true, maxSize) on each other one
Parity pins: see tests/test_oracle_*.py.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBS: dict = {}

F, U, T = 0, 1, 2

_KIND = {"cmp": 1, "between": 2, "in": 3, "codeset": 4, "isnull": 5, "notnull": 6,
         "and": 7, "or": 8, "not": 9, "isunknown": 10, "true": 11, "false": 12}
_CMP = {"=": 1, "<>": 2, "<": 3, "<=": 4, ">": 5, ">=": 6}
_WIDTH = {"i8": 1, "i16": 2, "i32": 4, "i64": 8}

NODE = np.dtype([("kind", "<i4"), ("col", "<i4"), ("cmp", "<i4"), ("nchild", "<i4"),
                 ("v1", "<i8"), ("v2", "<i8"), ("off", "<i8"), ("cnt", "<i8")])


class _Expr(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_void_p), ("root", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("children", ctypes.c_void_p), ("i64pool", ctypes.c_void_p),
                ("u32pool", ctypes.c_void_p)]


class _Col(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("data", ctypes.c_void_p), ("valid", ctypes.c_void_p)]


def load(path: str | None = None):
    """Load liboracle.so (or a given build of oracle.c; the environment
    variable SEL_ORACLE_LIB names another build, e.g. a sanitizer build)."""
    path = path or os.environ.get("SEL_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        from . import build as _b
        _b.build(out=path)
    L = ctypes.CDLL(path)
    vp, u64, i32, i64 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64
    L.oc_eval_row.argtypes = [vp, vp, u64]
    L.oc_eval_row.restype = ctypes.c_int
    L.oc_eval_all.argtypes = [vp, vp, u64, vp]
    L.oc_count.argtypes = [vp, vp, u64, ctypes.c_int]
    L.oc_count.restype = u64
    L.oc_rowids.argtypes = [vp, vp, u64, vp, u64]
    L.oc_rowids.restype = u64
    L.oc_rowids_mt.argtypes = [vp, vp, u64, vp, u64, ctypes.c_int]
    L.oc_rowids_mt.restype = u64
    L.oc_pushdown.argtypes = [vp, vp, u64, u64, vp, u64, vp]
    L.oc_pushdown.restype = ctypes.c_int
    L.oc_keybitmap.argtypes = [vp, vp, u64, i32, i64, vp, u64, vp]
    L.oc_keybitmap.restype = ctypes.c_int
    L.oc_star_count.argtypes = [vp, vp, u64, i32, vp, vp, vp, ctypes.c_int]
    L.oc_star_count.restype = u64
    _LIBS[path] = L
    return L


class Oracle:
    """Binds a table (datagen.Table) to one build of the oracle library."""

    def __init__(self, table, lib_path: str | None = None):
        self.lib = load(lib_path)
        self.table = table
        self._cols = (_Col * max(1, len(table.columns)))()
        self._keep = []
        for k, c in enumerate(table.columns):
            data = np.ascontiguousarray(c.data)
            self._keep.append(data)
            self._cols[k].width = _WIDTH[c.type]
            self._cols[k].data = data.ctypes.data
            if c.valid is not None:
                v = np.ascontiguousarray(c.valid, dtype=np.uint32)
                self._keep.append(v)
                self._cols[k].valid = v.ctypes.data
            else:
                self._cols[k].valid = None

    # ---- tree -> node array (the oracle's own representation) -------------
    def _expr(self, tree):
        nodes, children, i64, u32 = [], [], [], []

        def add(t):
            op = t[0]
            idx = len(nodes)
            nodes.append(None)
            rec = dict(kind=_KIND[op], col=0, cmp=0, nchild=0, v1=0, v2=0, off=0, cnt=0)
            if op == "cmp":
                rec.update(col=t[1], cmp=_CMP[t[2]], v1=_clamp64(t[3]))
                rec["_raw"] = t[3]
            elif op == "between":
                rec.update(col=t[1])
                rec["_lohi"] = (t[2], t[3])
            elif op == "in":
                rec.update(col=t[1], off=len(i64))
                vals = [v for v in t[2] if -(2 ** 63) <= v < 2 ** 63]
                i64.extend(vals)
                rec.update(cnt=len(vals))
            elif op == "codeset":
                words = np.asarray(t[3], dtype=np.uint32)
                rec.update(col=t[1], off=len(u32), cnt=int(t[2]))
                u32.extend(int(w) for w in words)
            elif op in ("isnull", "notnull"):
                rec.update(col=t[1])
            elif op in ("and", "or", "not", "isunknown"):
                kids = [add(k) for k in t[1:]]
                rec.update(off=len(children), nchild=len(kids))
                children.extend(kids)
            nodes[idx] = rec
            return idx

        root = add(tree)
        arr = np.zeros(len(nodes), dtype=NODE)
        for i, r in enumerate(nodes):
            # literals outside int64 cannot equal any value; express them exactly
            if r["kind"] == _KIND["cmp"]:
                raw = r.pop("_raw")
                r["kind"], r["cmp"], r["v1"], r["v2"] = _cmp_out_of_range(r["cmp"], raw)
            if r["kind"] == _KIND["between"]:
                lo, hi = r.pop("_lohi")
                if hi < lo or hi < -(2 ** 63) or lo > 2 ** 63 - 1:
                    r["v1"], r["v2"] = 1, 0          # empty interval: FALSE unless NULL
                else:
                    r["v1"], r["v2"] = max(lo, -(2 ** 63)), min(hi, 2 ** 63 - 1)
            for key in ("kind", "col", "cmp", "nchild", "v1", "v2", "off", "cnt"):
                arr[i][key] = r[key]
        ch = np.asarray(children if children else [0], dtype=np.int32)
        i64a = np.asarray(i64 if i64 else [0], dtype=np.int64)
        u32a = np.asarray(u32 if u32 else [0], dtype=np.uint32)
        e = _Expr(arr.ctypes.data, root, 0, ch.ctypes.data, i64a.ctypes.data, u32a.ctypes.data)
        return e, (arr, ch, i64a, u32a)

    # ---- queries -----------------------------------------------------------
    def eval_row(self, tree, row: int) -> int:
        e, keep = self._expr(tree)
        return self.lib.oc_eval_row(ctypes.byref(e), self._cols, row)

    def eval_all(self, tree) -> np.ndarray:
        e, keep = self._expr(tree)
        out = np.empty(self.table.nrows, dtype=np.uint8)
        self.lib.oc_eval_all(ctypes.byref(e), self._cols, self.table.nrows, out.ctypes.data)
        return out

    def count(self, tree, threads: int = 1) -> int:
        e, keep = self._expr(tree)
        return int(self.lib.oc_count(ctypes.byref(e), self._cols, self.table.nrows, threads))

    def rowids(self, tree, threads: int = 1) -> np.ndarray:
        """Ascending ids of the TRUE rows; threads > 1 splits the rows into
        contiguous ranges (oc_rowids_mt), one thread each."""
        e, keep = self._expr(tree)
        n = self.table.nrows
        if threads == 1:
            c = int(self.lib.oc_rowids(ctypes.byref(e), self._cols, n, None, 0))
            out = np.empty(c, dtype=np.uint32)
            self.lib.oc_rowids(ctypes.byref(e), self._cols, n, out.ctypes.data, c)
            return out
        c = int(self.lib.oc_rowids_mt(ctypes.byref(e), self._cols, n, None, 0, threads))
        out = np.empty(c, dtype=np.uint32)
        self.lib.oc_rowids_mt(ctypes.byref(e), self._cols, n, out.ctypes.data, c, threads)
        return out

    def pushdown(self, tree, max_rows: int, cap: int):
        """(status, count, ids) with status 0 OK, 1 over limit, 2 capacity."""
        e, keep = self._expr(tree)
        out = np.empty(max(1, min(cap, self.table.nrows)), dtype=np.uint32)
        cnt = ctypes.c_uint64(0)
        st = self.lib.oc_pushdown(ctypes.byref(e), self._cols, self.table.nrows, max_rows,
                                  out.ctypes.data, min(cap, out.size), ctypes.byref(cnt))
        c = int(cnt.value)
        if st == 0 and c > out.size:
            raise AssertionError("oracle capacity")
        return st, c, (out[:c].copy() if st == 0 else None)

    def keybitmap(self, tree, key_col: int, key_min: int, nbits: int):
        """(status, count, words) with status 0 or -6 (key out of range)."""
        e = keep = None
        if tree is not None:
            e, keep = self._expr(tree)
        words = np.zeros(max(1, (nbits + 31) // 32), dtype=np.uint32)
        cnt = ctypes.c_uint64(0)
        st = self.lib.oc_keybitmap(ctypes.byref(e) if e is not None else None, self._cols,
                                   self.table.nrows, key_col, key_min, words.ctypes.data,
                                   nbits, ctypes.byref(cnt))
        return st, int(cnt.value), words[: (nbits + 31) // 32]

    def star_count(self, fk_cols, bitmaps, nbits, tree=None, threads: int = 1) -> int:
        e = keep = None
        if tree is not None:
            e, keep = self._expr(tree)
        nfk = len(fk_cols)
        fk = np.asarray(fk_cols, dtype=np.int32)
        bms = [np.ascontiguousarray(b, dtype=np.uint32) for b in bitmaps]
        ptrs = (ctypes.c_void_p * nfk)(*[b.ctypes.data for b in bms])
        nb = np.asarray(nbits, dtype=np.uint64)
        return int(self.lib.oc_star_count(ctypes.byref(e) if e is not None else None,
                                          self._cols, self.table.nrows, nfk, fk.ctypes.data,
                                          ptrs, nb.ctypes.data, threads))


def and_factors(tree):
    """The conjuncts of a predicate tree: the operands of its top-level AND,
    nested ANDs flattened; the tree itself if its root is not an AND."""
    if tree[0] != "and":
        return [tree]
    out = []
    for t in tree[1:]:
        out += and_factors(t)
    return out


def factor_counts(table, tree, threads: int = 1):
    """(count of the selection, [count of each conjunct])."""
    orc = Oracle(table)
    return orc.count(tree, threads), [orc.count(f, threads) for f in and_factors(tree)]


def independence_estimate(nrows: int, counts) -> float:
    """|R| times the product of the conjuncts' selectivities: the estimate of
    a conjunction under the attribute-value independence assumption (the
    0.2 x 0.167 x 0.167 x 0.27 of Ch.1 sec.1.1)."""
    if nrows == 0:
        return 0.0
    e = float(nrows)
    for c in counts:
        e *= float(c) / float(nrows)
    return e


def q_error(estimate: float, exact: int) -> float:
    """max(estimate / exact, exact / estimate), both taken as at least 1 row."""
    e, x = max(float(estimate), 1.0), max(float(exact), 1.0)
    return max(e / x, x / e)


def join_size(r_rows, s_rows, v_r, v_s) -> float:
    """|R join S| on A = |R| |S| / max(V(R, A), V(S, A)), the simplified
    formula of Ch.1 sec.1.1 (V: distinct values of A)."""
    v = max(v_r, v_s)
    return r_rows * s_rows / v if v > 0 else 0.0


def star_plan_cost(fact_rows, dim_rows, sel_rows, order):
    """A left-deep plan joining the fact selection with the dimensions in
    `order`; the fact side holds every key of a dimension, the selected
    dimension sel_rows[d] of them.  (sum of intermediate sizes, sizes)."""
    cur, inter = float(fact_rows), []
    for d in order:
        cur = join_size(cur, sel_rows[d], dim_rows[d], sel_rows[d])
        inter.append(cur)
    return sum(inter), inter


def best_star_plan(fact_rows, dim_rows, sel_rows):
    """The cheapest left-deep order by trying every permutation (the first
    in lexicographic order among equal costs).  (order, cost)."""
    import itertools
    best = None
    for perm in itertools.permutations(range(len(dim_rows))):
        c, _ = star_plan_cost(fact_rows, dim_rows, sel_rows, perm)
        if best is None or c < best[1]:
            best = (list(perm), c)
    return best


def gather(table, ids, cols):
    """The projected columns of a materialised selection (Ch.3 sec.3.3):
    for each column index in `cols`, (values, valid) with values[k] the
    stored value at row ids[k] and valid[k] False where that row is NULL."""
    ids = np.asarray(ids, dtype=np.int64)
    out = []
    for c in cols:
        col = table.columns[c]
        vals = col.data[ids]
        if col.valid is None:
            valid = np.ones(ids.size, dtype=bool)
        else:
            valid = ((col.valid[ids >> 5] >> (ids & 31).astype(np.uint32)) & 1).astype(bool)
        out.append((vals, valid))
    return out


def max_size(nrows: int, ratio: float) -> int:
    """maxSize = R.size * PUSH_DOWN_MAX_SELECTIVITY (Algorithm 1), the product
    taken in double as the algorithm states it; an integer count exceeds it
    iff it exceeds its floor.  A ratio <= 0 (or NaN) gives 0, >= 1 gives
    nrows."""
    if not ratio > 0.0:
        return 0
    if ratio >= 1.0:
        return nrows
    return min(nrows, math.floor(float(nrows) * float(ratio)))


def select_pushdown(relations, min_table_size: int = 1000, max_selectivity: float = 0.05):
    """EvaluateAndPushDown of Algorithm 1 (Ch.4 sec.4.2), step by step.

    relations: [(table, tree or None[, cap])] -- a query's scanned relations,
    each with the selection extracted for it (None: no predicate on it) and
    optionally the capacity of the buffer its ids go to.  Returns one dict per
    relation, in input order: decision ('pushed', 'reverted', 'probe',
    'small', 'no_pred'), status (Execute's outcome for an evaluated relation:
    0 pushed, 1 count above maxSize, 2 above the capacity), order (position in
    the evaluation loop), count, max_rows and, for a pushed relation, its
    ascending row ids."""
    res = []
    for item in relations:
        t = item[0]
        res.append({"decision": None, "status": 0, "order": None, "count": 0,
                    "max_rows": max_size(t.nrows, max_selectivity), "ids": None})
    # the priority queue holds the relations larger than
    # PUSH_DOWN_MIN_TABLE_SIZE, by size, largest first; equal sizes keep the
    # order in which the scans were listed
    queue = []
    for i, item in enumerate(relations):
        if item[0].nrows > min_table_size:
            queue.append((item[0].nrows, i))
        else:
            res[i]["decision"] = "small"
    queue.sort(key=lambda e: (-e[0], e[1]))
    if not queue:
        return res
    # pop the largest relation: it is the one to be probed
    _, probe = queue.pop(0)
    res[probe]["decision"] = "probe"
    for k, (_, i) in enumerate(queue):
        t, tree = relations[i][0], relations[i][1]
        cap = relations[i][2] if len(relations[i]) > 2 else t.nrows
        res[i]["order"] = k
        if tree is None:
            res[i]["decision"] = "no_pred"
            continue
        # Execute(compound, true, maxSize): the exact count of sigma(R); a
        # count above maxSize throws and the push-down of R is reverted,
        # otherwise sigma(R) is materialised
        st, c, ids = Oracle(t).pushdown(tree, res[i]["max_rows"], cap)
        res[i]["status"] = st
        res[i]["count"] = c
        if st == 0:
            res[i]["decision"] = "pushed"
            res[i]["ids"] = ids
        else:
            res[i]["decision"] = "reverted"
    return res


def _clamp64(v: int) -> int:
    return max(-(2 ** 63), min(2 ** 63 - 1, int(v)))


def _cmp_out_of_range(cmp: int, v: int):
    """Comparison with an integer literal outside int64: no int64 value
    equals it, and every int64 value lies on one side of it.  Returns
    (kind, cmp, v1, v2) of an equivalent node on int64 literals."""
    lo, hi = -(2 ** 63), 2 ** 63 - 1
    if lo <= v <= hi:
        return _KIND["cmp"], cmp, v, 0
    below = v < lo          # every value is greater than v
    always = {  # truth for non-NULL rows
        _CMP["="]: False, _CMP["<>"]: True,
        _CMP["<"]: not below, _CMP["<="]: not below,
        _CMP[">"]: below, _CMP[">="]: below,
    }[cmp]
    if always:
        return _KIND["between"], 0, lo, hi      # TRUE for every non-NULL row
    return _KIND["between"], 0, 1, 0            # FALSE for every non-NULL row
