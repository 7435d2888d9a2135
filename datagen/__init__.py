"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module generates tables and predicate trees only; it evaluates no
predicate and counts nothing.  Columns come from ``libdatagen.so`` (counter
based SplitMix64 streams, identical for any thread count).  Predicate trees
are nested tuples in SQL terms; the product binding lowers them to its
postfix program and the oracle walks them directly:

    ('cmp', col, op, v)        op in '=', '<>', '<', '<=', '>', '>='
    ('between', col, lo, hi)   lo <= col <= hi
    ('in', col, (v, ...))
    ('codeset', col, nbits, words)   words: uint32 array, bit c = code c
    ('isnull', col) / ('notnull', col)
    ('and', p, q, ...) / ('or', p, q, ...) / ('not', p) / ('isunknown', p)
    ('true',) / ('false',)

``col`` is a column index.  Workload shapes follow the thesis' TPC-H/SSB
experiments (Ch.5): wide integer, DATE (day number), DECIMAL (scaled int64)
and dictionary-coded TEXT columns, with Zipf-skewed codes and NULLs.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

WIDTH = {"i8": 1, "i16": 2, "i32": 4, "i64": 8}
NP_DTYPE = {"i8": np.int8, "i16": np.int16, "i32": np.int32, "i64": np.int64}
TYPE_RANGE = {t: (int(np.iinfo(d).min), int(np.iinfo(d).max)) for t, d in NP_DTYPE.items()}


def lib():
    """Load libdatagen.so (built by datagen/build.py; the environment
    variable SEL_DATAGEN_LIB names another build, e.g. a sanitizer build)."""
    global _LIB
    if _LIB is None:
        path = os.environ.get("SEL_DATAGEN_LIB") or os.path.join(_HERE, "libdatagen.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        u64, i64, i32, vp, dbl = (ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                  ctypes.c_void_p, ctypes.c_double)
        L.dg_rand.argtypes = [u64, u64, u64]
        L.dg_rand.restype = u64
        L.dg_uniform.argtypes = [i32, u64, u64, i64, i64, vp, u64, i32]
        L.dg_zipf_cdf.argtypes = [dbl, u64, vp]
        L.dg_zipf.argtypes = [i32, u64, u64, vp, u64, vp, u64, i32]
        L.dg_lognormal_i64.argtypes = [u64, u64, dbl, dbl, vp, u64, i32]
        L.dg_validity.argtypes = [u64, u64, dbl, vp, u64, i32]
        L.dg_validity.restype = u64
        L.dg_fill_nulls.argtypes = [i32, vp, vp, u64, i64]
        L.dg_iota.argtypes = [i32, vp, u64, ctypes.c_uint32, i64]
        L.dg_code_bitmap.argtypes = [u64, u64, u64, vp, u64]
        L.dg_fnv1a.argtypes = [vp, u64]
        L.dg_fnv1a.restype = u64
        _LIB = L
    return _LIB


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Column:
    name: str
    type: str                      # 'i8' | 'i16' | 'i32' | 'i64'
    data: np.ndarray
    valid: np.ndarray | None = None  # uint32 words, bit i%32 of word i/32 = not NULL
    dict_card: int = 0
    null_count: int = 0


@dataclass
class Table:
    name: str
    nrows: int
    columns: list = field(default_factory=list)

    def index(self, name: str) -> int:
        for i, c in enumerate(self.columns):
            if c.name == name:
                return i
        raise KeyError(name)

    def col(self, name: str) -> Column:
        return self.columns[self.index(name)]

    def nbytes(self) -> int:
        n = 0
        for c in self.columns:
            n += c.data.nbytes + (c.valid.nbytes if c.valid is not None else 0)
        return n


# ---------------------------------------------------------------- columns --

def rand_u64(seed: int, stream: int, i: int) -> int:
    return int(lib().dg_rand(seed, stream, i))


def uniform(t: str, seed: int, stream: int, lo: int, hi: int, n: int, threads=None) -> np.ndarray:
    out = np.empty(n, dtype=NP_DTYPE[t])
    lib().dg_uniform(WIDTH[t], seed, stream, lo, hi, _ptr(out), n, threads or default_threads())
    return out


def zipf(t: str, seed: int, stream: int, s: float, ncodes: int, n: int, threads=None) -> np.ndarray:
    cdf = np.empty(ncodes, dtype=np.float64)
    lib().dg_zipf_cdf(s, ncodes, _ptr(cdf))
    out = np.empty(n, dtype=NP_DTYPE[t])
    lib().dg_zipf(WIDTH[t], seed, stream, _ptr(cdf), ncodes, _ptr(out), n,
                  threads or default_threads())
    return out


def zipf_pmf(s: float, ncodes: int) -> np.ndarray:
    """Probability of code c (= rank c+1) under Zipf(s) over ncodes ranks."""
    w = np.arange(1, ncodes + 1, dtype=np.float64) ** (-s)
    return w / w.sum()


def lognormal_i64(seed: int, stream: int, mu: float, sigma: float, n: int, threads=None):
    out = np.empty(n, dtype=np.int64)
    lib().dg_lognormal_i64(seed, stream, mu, sigma, _ptr(out), n, threads or default_threads())
    return out


def validity(seed: int, stream: int, rate: float, n: int, threads=None):
    words = np.empty((n + 31) // 32, dtype=np.uint32)
    nulls = lib().dg_validity(seed, stream, rate, _ptr(words), n, threads or default_threads())
    return words, int(nulls)


def fill_nulls(col: Column, value: int) -> None:
    lib().dg_fill_nulls(WIDTH[col.type], _ptr(col.data), _ptr(col.valid), col.data.size, value)


def iota(t: str, n: int, shift: int = 0, base: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=NP_DTYPE[t])
    lib().dg_iota(WIDTH[t], _ptr(out), n, shift, base)
    return out


def code_bitmap(seed: int, stream: int, mod: int, nbits: int) -> np.ndarray:
    words = np.empty((nbits + 31) // 32, dtype=np.uint32)
    lib().dg_code_bitmap(seed, stream, mod, _ptr(words), nbits)
    return words


def checksum(a: np.ndarray) -> int:
    a = np.ascontiguousarray(a)
    return int(lib().dg_fnv1a(_ptr(a), a.nbytes))


def words_from_codes(codes, nbits: int) -> np.ndarray:
    words = np.zeros((nbits + 31) // 32, dtype=np.uint32)
    for c in codes:
        words[c // 32] |= np.uint32(1 << (c % 32))
    return words


# ---------------------------------------------------------------- configs --

def cfg1(n: int = 1_000_000, seed: int = 1, threads=None) -> Table:
    """One table of three int32 columns uniform in [0, 10000)."""
    t = Table("cfg1", n)
    for k in range(3):
        t.columns.append(Column(f"c{k}", "i32", uniform("i32", seed, k, 0, 9999, n, threads)))
    return t


def cfg1_predicate():
    """c0 < 3000 AND c1 BETWEEN 3500 AND 6499 AND c2 >= 7000 (each ~30 %)."""
    return ("and", ("cmp", 0, "<", 3000), ("between", 1, 3500, 6499), ("cmp", 2, ">=", 7000))


CFG2_COLUMNS = ["date", "qty", "disc", "price", "s7", "s25", "s4500", "okey"]
CFG2_NULL_RATE = 0.05
CFG2_PRICE_NULL_FILL = 1_000_000   # a value that satisfies price >= 20000


def lineorder_like(name: str, n: int, seed: int, threads=None) -> Table:
    """Fact table with TPC-H/SSB-like columns: DATE as a day number over 2557
    days, int8 quantity 1..50 and discount 0..10, DECIMAL price as log-normal
    int64 with 5 % NULLs, three dictionary-coded TEXT columns (Zipf 1.1 over
    7, 25 and 4500 codes) and an unreferenced int32 order key."""
    t = Table(name, n)
    t.columns.append(Column("date", "i32", uniform("i32", seed, 0, 0, 2556, n, threads)))
    t.columns.append(Column("qty", "i8", uniform("i8", seed, 1, 1, 50, n, threads)))
    t.columns.append(Column("disc", "i8", uniform("i8", seed, 2, 0, 10, n, threads)))
    price = Column("price", "i64", lognormal_i64(seed, 3, 10.0, 1.0, n, threads))
    price.valid, price.null_count = validity(seed, 4, CFG2_NULL_RATE, n, threads)
    fill_nulls(price, CFG2_PRICE_NULL_FILL)
    t.columns.append(price)
    for k, card in zip((5, 6, 7), (7, 25, 4500)):
        t.columns.append(Column(f"s{card}", "i32", zipf("i32", seed, k, 1.1, card, n, threads),
                                dict_card=card))
    t.columns.append(Column("okey", "i32", iota("i32", n, shift=2)))
    return t


def cfg2(n: int = 300_000_000, seed: int = 2, threads=None) -> Table:
    return lineorder_like("cfg2", n, seed, threads)


def sparse_in_values(col: np.ndarray, k: int, seed: int = 95, absent_lo: int = 10**7,
                     absent_hi: int = 10**8) -> tuple:
    """An IN list of k values too sparse for a bitmap: half drawn from the
    first 10 M rows of `col` (so they occur), half from [absent_lo,
    absent_hi) (above the log-normal price column's values), as a tuple."""
    rng = np.random.default_rng(seed + k)
    present = rng.choice(col[:10_000_000], k // 2, replace=False)
    absent = rng.integers(absent_lo, absent_hi, k - k // 2)
    return tuple(int(v) for v in np.concatenate([present, absent]))


def cfg2_like_bitmap(seed: int = 6) -> np.ndarray:
    """A LIKE pattern on s4500 resolved to codes: bit c set iff
    rand(seed, 0, c) % 8 == 0."""
    return code_bitmap(seed, 0, 8, 4500)


def cfg2_predicate(date_lo: int = 365, date_hi: int = 729):
    """date BETWEEN lo AND hi AND (qty < 25 OR disc BETWEEN 5 AND 7) AND
    (price >= 20000 OR s25 IN (0,2,...,18)) AND s4500 LIKE <pattern>."""
    return ("and",
            ("between", 0, date_lo, date_hi),
            ("or", ("cmp", 1, "<", 25), ("between", 2, 5, 7)),
            ("or", ("cmp", 3, ">=", 20000), ("in", 5, tuple(range(0, 20, 2)))),
            ("codeset", 6, 4500, cfg2_like_bitmap()))


# ---- star schema: fact table with foreign keys into four dimensions --------

CFG4_DIM_ROWS = (2556, 30_000, 200_000, 3_200_000)


def star_dims(seed: int = 42, sizes=CFG4_DIM_ROWS, threads=None):
    """Dimension tables with a dense int32 primary key (= row index) and
    low-cardinality, partly hierarchical attributes."""
    d0n, d1n, d2n, d3n = sizes
    dims = []
    # dates: key, year (day/365), month-of-year
    d0 = Table("d_date", d0n)
    d0.columns.append(Column("key", "i32", iota("i32", d0n)))
    year = (np.arange(d0n, dtype=np.int64) // 365).astype(np.int32)
    d0.columns.append(Column("year", "i32", year, dict_card=int(year.max()) + 1))
    d0.columns.append(Column("month", "i32", ((np.arange(d0n) % 365) // 31).astype(np.int32),
                             dict_card=12))
    dims.append(d0)
    # customers: key, region (5), nation = region*5 + U{0..4}
    d1 = Table("d_customer", d1n)
    d1.columns.append(Column("key", "i32", iota("i32", d1n)))
    region = uniform("i32", seed, 0, 0, 4, d1n, threads)
    d1.columns.append(Column("region", "i32", region, dict_card=5))
    d1.columns.append(Column("nation", "i32",
                             region * 5 + uniform("i32", seed, 1, 0, 4, d1n, threads),
                             dict_card=25))
    dims.append(d1)
    # parts: key, category (25), brand = category*40 + U{0..39}
    d2 = Table("d_part", d2n)
    d2.columns.append(Column("key", "i32", iota("i32", d2n)))
    cat = uniform("i32", seed + 1, 0, 0, 24, d2n, threads)
    d2.columns.append(Column("category", "i32", cat, dict_card=25))
    d2.columns.append(Column("brand", "i32",
                             cat * 40 + uniform("i32", seed + 1, 1, 0, 39, d2n, threads),
                             dict_card=1000))
    dims.append(d2)
    # suppliers: key, city (250), nation = city // 10
    d3 = Table("d_supplier", d3n)
    d3.columns.append(Column("key", "i32", iota("i32", d3n)))
    city = uniform("i32", seed + 2, 0, 0, 249, d3n, threads)
    d3.columns.append(Column("city", "i32", city, dict_card=250))
    d3.columns.append(Column("nation", "i32", city // 10, dict_card=25))
    dims.append(d3)
    return dims


def star_dim_predicates():
    """One predicate per dimension, selectivities about 2/7, 1/5, 2/25, 8/1000."""
    return [
        ("in", 1, (1, 2)),                                    # year IN (1, 2)
        ("cmp", 1, "=", 2),                                   # region = 2
        ("or", ("cmp", 1, "=", 3), ("cmp", 1, "=", 7)),       # category 3 or 7
        ("in", 1, (17, 101)),                                 # two cities
    ]


def star_fact(n: int = 480_000_000, seed: int = 41, dim_rows=CFG4_DIM_ROWS, threads=None):
    """Fact table: fk0..fk3 int32 uniform over the dimension keys, m0..m2
    int32 measures."""
    t = Table("fact", n)
    for d, rows in enumerate(dim_rows):
        t.columns.append(Column(f"fk{d}", "i32", uniform("i32", seed, d, 0, rows - 1, n, threads)))
    t.columns.append(Column("m0", "i32", uniform("i32", seed, 4, 1, 50, n, threads)))
    t.columns.append(Column("m1", "i32", uniform("i32", seed, 5, 0, 99, n, threads)))
    t.columns.append(Column("m2", "i32", uniform("i32", seed, 6, 0, 1_000_000, n, threads)))
    return t


def star_fact_predicate():
    """Optional fact-side predicate: m1 < 50."""
    return ("cmp", 5, "<", 50)


# ---- batching: many candidate predicates over tables of uneven size --------

CFG3_ROWS = (10_000, 2_000_000, 60_000_000, 300_000_000)
CFG3_SEEDS = (31, 32, 33, 34)


def cfg3_tables(rows=CFG3_ROWS, threads=None):
    """Four tables with the fact-table schema (seeds 31..34)."""
    return [lineorder_like(f"T{k}", n, seed, threads)
            for k, (n, seed) in enumerate(zip(rows, CFG3_SEEDS))]


def _inv_norm_sf(q: float) -> float:
    """z with P(Z >= z) = q for a standard normal (bisection on erfc)."""
    lo, hi = -40.0, 40.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 0.5 * math.erfc(mid / math.sqrt(2.0)) > q:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _leaf_for(rng: np.random.Generator, q: float):
    """A leaf over the fact-table schema whose selectivity is about q, set
    from the column's known marginal distribution."""
    q = min(max(q, 1e-7), 1.0)
    col = int(rng.choice([0, 1, 2, 3, 5, 6]))
    if col == 0:                                  # date uniform over 2557 days
        w = max(1, int(round(q * 2557)))
        a = int(rng.integers(0, 2557 - w + 1))
        return ("between", 0, a, a + w - 1)
    if col == 1:                                  # qty uniform 1..50
        w = max(1, int(round(q * 50)))
        return ("cmp", 1, "<", 1 + w) if rng.random() < 0.5 else ("cmp", 1, ">", 50 - w)
    if col == 2:                                  # disc uniform 0..10
        w = max(1, int(round(q * 11)))
        a = int(rng.integers(0, 11 - w + 1))
        return ("between", 2, a, a + w - 1)
    if col == 3:                                  # price log-normal(10, 1)
        v = int(round(math.exp(10.0 + _inv_norm_sf(q))))
        return ("cmp", 3, ">=", v)
    card = 25 if col == 5 else 4500               # Zipf(1.1) dictionary codes
    pmf = zipf_pmf(1.1, card)
    order = rng.permutation(card)
    codes, mass = [], 0.0
    for c in order:
        if mass >= q:
            break
        if mass + pmf[c] > q * 1.5 and codes:
            continue
        codes.append(int(c))
        mass += pmf[c]
    if col == 5:
        return ("in", 5, tuple(sorted(codes)))
    return ("codeset", 6, 4500, words_from_codes(codes, 4500))


def cfg3_programs(seed: int = 35, per_table: int = 16, ntables: int = 4):
    """Candidate predicates: for each table, per_table programs with 2..8
    leaves and target selectivity log-uniform in [1e-5, 0.9]; each is an AND
    of m factors of selectivity about s^(1/m), some factors 2-leaf ORs.
    Returns a list of (table index, tree)."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(ntables):
        for _ in range(per_table):
            k = int(rng.integers(2, 9))
            s = math.exp(rng.uniform(math.log(1e-5), math.log(0.9)))
            n_or = int(rng.integers(0, k // 2 + 1))
            m = k - n_or
            q = s ** (1.0 / m)
            factors = []
            for f in range(m):
                if f < n_or:
                    q2 = 1.0 - math.sqrt(max(0.0, 1.0 - q))
                    factors.append(("or", _leaf_for(rng, q2), _leaf_for(rng, q2)))
                else:
                    factors.append(_leaf_for(rng, q))
            tree = factors[0] if m == 1 else ("and", *factors)
            out.append((t, tree))
    return out


# ---- serving: a Poisson stream of estimate requests --------------------------

SERVE_TABLES = ("cfg1_1M", "T_2M", "T_60M", "fact_300M", "star_480M")


def uniform3_programs(seed: int, n: int):
    """Programs over three int32 columns uniform in [0, 10000): ANDs of 1..3
    range leaves with per-leaf selectivity log-uniform in [1e-3, 0.9]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        k = int(rng.integers(1, 4))
        leaves = []
        for c in rng.permutation(3)[:k]:
            q = math.exp(rng.uniform(math.log(1e-3), math.log(0.9)))
            w = max(1, int(round(q * 10000)))
            a = int(rng.integers(0, 10000 - w + 1))
            leaves.append(("between", int(c), a, a + w - 1))
        out.append(leaves[0] if k == 1 else ("and", *leaves))
    return out


def star_dim_programs(seed: int, n: int, dims):
    """n combinations of one predicate per dimension (on its non-key
    attributes), with selectivities spread over orders of magnitude."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        combo = []
        for d in dims:
            col = int(rng.integers(1, len(d.columns)))
            card = d.columns[col].dict_card
            k = max(1, int(round(card * math.exp(rng.uniform(math.log(0.02), math.log(0.6))))))
            codes = tuple(sorted(int(c) for c in rng.choice(card, size=min(k, card), replace=False)))
            combo.append(("in", col, codes))
        out.append(combo)
    return out


def serving_trace(seed: int = 52, rate: float = 2000.0, duration: float = 10.0,
                  pool_sizes=(32, 32, 32, 32, 16), pushdown_rate: float = 0.1,
                  max_programs: int = 12):
    """Poisson arrivals (rate per second over `duration` seconds); each
    request has 1..max_programs programs, each on a table drawn uniformly
    from the five resident tables and a program drawn from that table's
    pool; a fraction asks, in addition, for one push-down with row ids on a
    non-star table.  Returns [(arrival_s, [(table, prog)], pushdown)] with
    pushdown None or (table, prog)."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        k = int(rng.integers(1, max_programs + 1))
        items = []
        for _ in range(k):
            tb = int(rng.integers(0, len(pool_sizes)))
            items.append((tb, int(rng.integers(0, pool_sizes[tb]))))
        pd = None
        if rng.random() < pushdown_rate:
            tb = int(rng.integers(0, len(pool_sizes) - 1))
            pd = (tb, int(rng.integers(0, pool_sizes[tb])))
        out.append((t, items, pd))
    return out


# ---------------------------------------------------- random tiny inputs --

def grid_values(t: str):
    lo, hi = TYPE_RANGE[t]
    return [lo, lo + 1, -1, 0, 1, 2, hi - 1, hi]


def random_table(rng: np.random.Generator, n: int, types=("i8", "i16", "i32", "i64"),
                 null_rate=0.2, grid=True, name="rand") -> Table:
    """Small table whose values come from tiny grids (type extremes, -1, 0,
    1, 2) or small uniform ranges, with random NULLs."""
    t = Table(name, n)
    for k, ty in enumerate(types):
        if grid:
            vals = np.array(grid_values(ty), dtype=NP_DTYPE[ty])
            data = vals[rng.integers(0, len(vals), n)]
        else:
            data = rng.integers(-20, 21, n).astype(NP_DTYPE[ty])
        # dictionary-coded (so code-set tests apply); most grid values are
        # outside [0, dict_card), which a code-set test treats as FALSE
        col = Column(f"x{k}", ty, np.ascontiguousarray(data), dict_card=64)
        if null_rate > 0 and rng.random() < 0.75:
            isnull = rng.random(n) < null_rate
            words = np.zeros((n + 31) // 32, dtype=np.uint32)
            bits = np.packbits((~isnull).astype(np.uint8), bitorder="little")
            buf = np.zeros(words.size * 4, dtype=np.uint8)
            buf[: bits.size] = bits
            words = buf.view(np.uint32).copy()
            col.valid = words
            col.null_count = int(isnull.sum())
        t.columns.append(col)
    return t


def random_leaf(rng: np.random.Generator, table: Table, grid=True):
    k = int(rng.integers(0, len(table.columns)))
    col = table.columns[k]
    pool = grid_values(col.type) if grid else list(range(-21, 22))
    lo_t, hi_t = TYPE_RANGE[col.type]
    # literals may lie outside the column type (folded by the compiler)
    extra = [lo_t - 1, hi_t + 1, -(2 ** 63), 2 ** 63 - 1]
    choice = lambda: int(rng.choice(pool + extra if rng.random() < 0.2 else pool))
    kind = rng.choice(["cmp", "between", "in", "codeset", "isnull", "notnull"],
                      p=[0.4, 0.2, 0.15, 0.1, 0.075, 0.075])
    if kind == "cmp":
        return ("cmp", k, str(rng.choice(["=", "<>", "<", "<=", ">", ">="])), choice())
    if kind == "between":
        a, b = choice(), choice()
        if rng.random() < 0.7 and a > b:
            a, b = b, a
        return ("between", k, a, b)
    if kind == "in":
        m = int(rng.integers(1, 6))
        return ("in", k, tuple(choice() for _ in range(m)))
    if kind == "codeset":
        nbits = int(rng.integers(1, 70))
        codes = [int(c) for c in rng.integers(0, nbits, int(rng.integers(0, nbits + 1)))]
        return ("codeset", k, nbits, words_from_codes(codes, nbits))
    return (str(kind), k)


def random_tree(rng: np.random.Generator, table: Table, max_depth=6, max_leaves=12, grid=True):
    """Random predicate tree over `table` (depth <= max_depth, leaves <=
    max_leaves), mixing AND / OR / NOT / IS UNKNOWN and constants."""
    budget = [max_leaves]

    def gen(depth):
        if depth >= max_depth or budget[0] <= 1 or rng.random() < 0.35:
            budget[0] -= 1
            r = rng.random()
            if r < 0.03:
                return ("true",)
            if r < 0.06:
                return ("false",)
            return random_leaf(rng, table, grid)
        r = rng.random()
        if r < 0.15:
            return ("not", gen(depth + 1))
        if r < 0.22:
            return ("isunknown", gen(depth + 1))
        op = "and" if r < 0.62 else "or"
        m = int(rng.integers(2, 4))
        kids = []
        for _ in range(m):
            if budget[0] <= 0:
                break
            kids.append(gen(depth + 1))
        if len(kids) < 2:
            return kids[0] if kids else random_leaf(rng, table, grid)
        return (op, *kids)

    return gen(0)


def tree_leaves(tree) -> int:
    if tree[0] in ("and", "or"):
        return sum(tree_leaves(k) for k in tree[1:])
    if tree[0] in ("not", "isunknown"):
        return tree_leaves(tree[1])
    return 1


def tree_columns(tree) -> set:
    if tree[0] in ("and", "or", "not", "isunknown"):
        s = set()
        for k in tree[1:]:
            s |= tree_columns(k)
        return s
    if tree[0] in ("true", "false"):
        return set()
    return {tree[1]}
