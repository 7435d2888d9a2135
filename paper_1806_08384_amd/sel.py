"""ctypes binding of libsel (include/sel.h): argument marshalling only.

Every step of the path runs in libsel's HIP kernels; this module converts
Python values to the C ABI and back.  Predicate trees (nested tuples in SQL
terms, see ``datagen``) are flattened to the ABI's postfix ``sel_instr``
program plus its constant pool; all lowering happens in the library.

If libsel.so is missing or cannot be loaded this module raises at import:
there is no CPU fallback.
"""
from __future__ import annotations

import collections
import ctypes
import os
import weakref

import numpy as np
# torch first: its HIP runtime (soname libamdhip64.so.7) is then the one
# libsel binds to, so the process holds a single HIP runtime and both share
# devices, streams and memory.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsel.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1806_08384_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# ---- ABI constants (include/sel.h) -----------------------------------------
SEL_OK, SEL_OVER_LIMIT, SEL_E_CAPACITY = 0, 1, 2
SEL_E_INVALID, SEL_E_TYPE, SEL_E_NOMEM, SEL_E_DEVICE, SEL_E_BUSY, SEL_E_RANGE = -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "SEL_OK", 1: "SEL_OVER_LIMIT", 2: "SEL_E_CAPACITY", -1: "SEL_E_INVALID",
                -2: "SEL_E_TYPE", -3: "SEL_E_NOMEM", -4: "SEL_E_DEVICE", -5: "SEL_E_BUSY",
                -6: "SEL_E_RANGE"}
TYPES = {"i8": 1, "i16": 2, "i32": 3, "i64": 4}
OP = {"=": 1, "<>": 2, "<": 3, "<=": 4, ">": 5, ">=": 6, "between": 7, "in": 8, "codeset": 9,
      "isnull": 10, "notnull": 11, "and": 16, "or": 17, "not": 18, "isunknown": 19,
      "true": 20, "false": 21}
K_COUNT, K_MASK, K_SCAN, K_COMPACT, K_KEYBITMAP, K_STAR, K_BATCH, K_GATHER, K_NKINDS = range(9)
INT64_MIN, INT64_MAX = -(2 ** 63), 2 ** 63 - 1
UINT64_MAX = 2 ** 64 - 1


class SelError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sel_column(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("dict_card", ctypes.c_uint32),
                ("data", ctypes.c_void_p), ("valid", ctypes.c_void_p)]


class sel_instr(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint16), ("col", ctypes.c_uint16), ("aux", ctypes.c_uint32),
                ("a", ctypes.c_int64), ("b", ctypes.c_int64)]


class sel_launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_uint32), ("grid", ctypes.c_uint32), ("cached", ctypes.c_uint32),
                ("tiles_per_step", ctypes.c_uint32), ("stage_words", ctypes.c_uint32),
                ("rows_per_lane", ctypes.c_uint32)]


Launch = collections.namedtuple("Launch", "block grid cached tiles_per_step stage_words rows_per_lane")


def _launch(l: sel_launch) -> Launch:
    return Launch(l.block, l.grid, l.cached, l.tiles_per_step, l.stage_words, l.rows_per_lane)


class sel_spd_relation(ctypes.Structure):
    _fields_ = [("table", ctypes.c_void_p), ("pred", ctypes.c_void_p), ("d_out", ctypes.c_void_p),
                ("cap", ctypes.c_uint64)]


class sel_spd_result(ctypes.Structure):
    _fields_ = [("decision", ctypes.c_int32), ("status", ctypes.c_int32), ("order", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("count", ctypes.c_uint64), ("max_rows", ctypes.c_uint64)]


SPD_DECISIONS = ("pushed", "reverted", "probe", "small", "no_pred")


class sel_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("chunk_rows", ctypes.c_uint64),
                ("max_programs", ctypes.c_uint32), ("rounds_in_flight", ctypes.c_uint32),
                ("rounds_per_cycle", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class sel_request(ctypes.Structure):
    _fields_ = [("nprog", ctypes.c_uint32), ("tables", ctypes.POINTER(ctypes.c_void_p)),
                ("progs", ctypes.POINTER(ctypes.c_void_p)), ("pd_table", ctypes.c_void_p),
                ("pd_prog", ctypes.c_void_p), ("pd_max_rows", ctypes.c_uint64),
                ("pd_out", ctypes.c_void_p), ("pd_cap", ctypes.c_uint64)]


class sel_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("pad", ctypes.c_int32), ("pd_count", ctypes.c_uint64),
                ("latency_ms", ctypes.c_double)]


class sel_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("rounds", ctypes.c_uint64),
                ("round_programs", ctypes.c_uint64), ("shared_rounds", ctypes.c_uint64),
                ("max_admitted", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
                ("elapsed_s", ctypes.c_double), ("round_groups", ctypes.c_uint64),
                ("round_gpu_ms", ctypes.c_double), ("round_host_ms", ctypes.c_double),
                ("round_bytes", ctypes.c_double)]


class sel_timing(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * K_NKINDS), ("launches", ctypes.c_uint64 * K_NKINDS)]


_vp, _u64, _u32, _i32, _i64 = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                               ctypes.c_int32, ctypes.c_int64)
_P = ctypes.POINTER


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


sel_ctx_create = _sig("sel_ctx_create", _i32, ctypes.c_int, _vp, _P(_vp))
sel_ctx_destroy = _sig("sel_ctx_destroy", None, _vp)
sel_last_error = _sig("sel_last_error", ctypes.c_char_p, _vp)
sel_ctx_num_cus = _sig("sel_ctx_num_cus", _u32, _vp)
sel_table_create = _sig("sel_table_create", _i32, _vp, _u64, _u32, _P(sel_column), _P(_vp))
sel_table_destroy = _sig("sel_table_destroy", None, _vp)
sel_table_nrows = _sig("sel_table_nrows", _u64, _vp)
sel_program_compile = _sig("sel_program_compile", _i32, _vp, _vp, _P(sel_instr), _u32, _vp, _u32,
                           _P(_vp))
sel_program_destroy = _sig("sel_program_destroy", None, _vp)
sel_program_check = _sig("sel_program_check", _i32, _u64, _u32, _P(sel_column), _P(sel_instr), _u32,
                         _vp, _u32, ctypes.c_char_p, ctypes.c_size_t, ctypes.c_char_p,
                         ctypes.c_size_t)
sel_program_listing = _sig("sel_program_listing", ctypes.c_char_p, _vp)
sel_program_bytes_per_row = _sig("sel_program_bytes_per_row", ctypes.c_double, _vp)
sel_count = _sig("sel_count", _i32, _vp, _vp, _vp, _P(_u64))
sel_count_async = _sig("sel_count_async", _i32, _vp, _vp, _vp, _vp)
sel_max_rows = _sig("sel_max_rows", _u64, _u64, ctypes.c_double)
sel_pushdown_rowids = _sig("sel_pushdown_rowids", _i32, _vp, _vp, _vp, _u64, _vp, _u64, _P(_u64))
sel_pushdown_rowids_noalloc = _sig("sel_pushdown_rowids_noalloc", _i32, _vp, _vp, _vp, _u64, _vp, _u64,
                                   _P(_u64))
sel_pushdown_keybitmap = _sig("sel_pushdown_keybitmap", _i32, _vp, _vp, _u32, _i64, _vp, _vp, _u64,
                              _P(_u64))
sel_star_count = _sig("sel_star_count", _i32, _vp, _vp, _vp, _u32, _P(_u32), _P(_vp), _P(_u64),
                      _P(_u64))
sel_count_batch = _sig("sel_count_batch", _i32, _vp, _u32, _P(_vp), _P(_vp), _P(_u64))
sel_factor_counts = _sig("sel_factor_counts", _i32, _vp, _vp, _vp, _u32, _P(_u64), _P(_u32), _P(_u64))
sel_independence_estimate = _sig("sel_independence_estimate", ctypes.c_double, _u64, _u32, _P(_u64))
sel_join_size = _sig("sel_join_size", ctypes.c_double, ctypes.c_double, ctypes.c_double,
                     ctypes.c_double, ctypes.c_double)
sel_star_plan_cost = _sig("sel_star_plan_cost", ctypes.c_double, ctypes.c_double, _u32,
                          _P(ctypes.c_double), _P(ctypes.c_double), _P(_u32), _P(ctypes.c_double))
sel_star_plan_order = _sig("sel_star_plan_order", _i32, ctypes.c_double, _u32, _P(ctypes.c_double),
                           _P(ctypes.c_double), _P(_u32), _P(ctypes.c_double))
sel_gather = _sig("sel_gather", _i32, _vp, _vp, _vp, _u64, _u32, _P(_u32), _P(_vp), _P(_vp))
sel_select_pushdown = _sig("sel_select_pushdown", _i32, _vp, _u32, _P(sel_spd_relation), _u64,
                           ctypes.c_double, _P(sel_spd_result))
sel_batch_create = _sig("sel_batch_create", _i32, _vp, _u32, _P(_vp), _P(_vp), _P(_vp))
sel_batch_set_program = _sig("sel_batch_set_program", _i32, _vp, _u32, _vp)
sel_batch_run = _sig("sel_batch_run", _i32, _vp, _P(_u64))
sel_batch_destroy = _sig("sel_batch_destroy", None, _vp)
sel_autotune = _sig("sel_autotune", _i32, _vp, _vp, _vp, ctypes.c_int, _u32, _P(sel_launch),
                    _P(ctypes.c_double))
sel_autotune_batch = _sig("sel_autotune_batch", _i32, _vp, _u32, _P(_vp), _P(_vp), _u32,
                          _P(sel_launch), _P(ctypes.c_double))
sel_tune_save = _sig("sel_tune_save", _i32, _vp, ctypes.c_char_p)
sel_tune_load = _sig("sel_tune_load", _i32, _vp, ctypes.c_char_p)
sel_tune_entries = _sig("sel_tune_entries", _u32, _vp)
sel_program_star = _sig("sel_program_star", _i32, _vp, _vp, _vp, _u32, _P(_u32), _P(_vp), _P(_u64),
                        _P(_vp))
sel_server_create = _sig("sel_server_create", _i32, _vp, _P(sel_server_config), _P(_vp))
sel_server_submit = _sig("sel_server_submit", _i32, _vp, _P(sel_request), _P(_u64))
sel_server_poll = _sig("sel_server_poll", _i32, _vp, _u64, _P(ctypes.c_int))
sel_server_wait = _sig("sel_server_wait", _i32, _vp, _u64, _P(_u64), _P(sel_result))
sel_server_get_stats = _sig("sel_server_get_stats", _i32, _vp, _P(sel_server_stats), ctypes.c_int)
sel_server_destroy = _sig("sel_server_destroy", None, _vp)
sel_ctx_set_launch = _sig("sel_ctx_set_launch", _i32, _vp, _P(sel_launch))
sel_ctx_enable_timing = _sig("sel_ctx_enable_timing", _i32, _vp, ctypes.c_int)
sel_ctx_read_timing = _sig("sel_ctx_read_timing", _i32, _vp, _P(sel_timing), ctypes.c_int)

EXPORTED = [n for n in list(globals()) if n.startswith("sel_") and callable(globals()[n])
            and hasattr(globals()[n], "argtypes")]


# ---- predicate tree -> postfix program + pool ----------------------------------

def _lit(v) -> int:
    v = int(v)
    if not INT64_MIN <= v <= INT64_MAX:
        raise ValueError(f"literal {v} outside int64 (the ABI takes int64 literals)")
    return v


def flatten(tree):
    """Postfix sel_instr array and pool bytes for a predicate tree."""
    code: list = []
    pool = bytearray()

    def put(op, col=0, aux=0, a=0, b=0):
        code.append((OP[op], col, aux, a, b))

    def align(n):
        while len(pool) % n:
            pool.append(0)

    def walk(t):
        k = t[0]
        if k == "cmp":
            put(t[2], t[1], 0, _lit(t[3]))
        elif k == "between":
            put("between", t[1], 0, _lit(t[2]), _lit(t[3]))
        elif k == "in":
            vals = np.asarray([_lit(v) for v in t[2]], dtype=np.int64)
            align(8)
            off = len(pool)
            pool.extend(vals.tobytes())
            put("in", t[1], off, 0, len(vals))
        elif k == "codeset":
            words = np.ascontiguousarray(t[3], dtype=np.uint32)
            align(4)
            off = len(pool)
            pool.extend(words.tobytes())
            put("codeset", t[1], off, 0, int(t[2]))
        elif k in ("isnull", "notnull"):
            put(k, t[1])
        elif k in ("true", "false"):
            put(k)
        elif k in ("not", "isunknown"):
            walk(t[1])
            put(k)
        elif k in ("and", "or"):
            walk(t[1])
            for c in t[2:]:
                walk(c)
                put(k)
        else:
            raise ValueError(f"unknown node {k!r}")

    walk(tree)
    arr = (sel_instr * len(code))()
    for i, (op, col, aux, a, b) in enumerate(code):
        arr[i].op, arr[i].col, arr[i].aux, arr[i].a, arr[i].b = op, col, aux, a, b
    return arr, bytes(pool)


def _columns_struct(cols):
    arr = (sel_column * len(cols))()
    for i, (ty, card, data, valid) in enumerate(cols):
        arr[i].type = TYPES[ty] if isinstance(ty, str) else int(ty)
        arr[i].dict_card = card
        arr[i].data = data
        arr[i].valid = valid
    return arr


def check_program(nrows: int, col_specs, tree):
    """Host-only validation + lowering (sel_program_check): returns
    (status, listing, error) without any device work.  col_specs: list of
    (type, dict_card, nullable)."""
    cols = _columns_struct([(ty, card, None, 8 if nullable else None)
                            for ty, card, nullable in col_specs])
    code, pool = flatten(tree)
    return check_raw(nrows, cols, code, pool)


def check_raw(nrows, cols, code, pool: bytes):
    text = ctypes.create_string_buffer(16384)
    err = ctypes.create_string_buffer(512)
    pbuf = ctypes.create_string_buffer(pool, max(1, len(pool)))
    st = sel_program_check(nrows, len(cols), cols, code, len(code), pbuf, len(pool), text,
                           len(text), err, len(err))
    return st, text.value.decode(), err.value.decode()


# ---- object wrappers -------------------------------------------------------------

def join_size(r_rows, s_rows, v_r, v_s) -> float:
    return float(sel_join_size(r_rows, s_rows, v_r, v_s))


def star_plan(fact_rows, dim_rows, sel_rows, order=None):
    """(order, cost, intermediate sizes) of a left-deep star plan: the given
    order, or the library's cheapest one."""
    n = len(dim_rows)
    dr = (ctypes.c_double * max(1, n))(*dim_rows)
    sr = (ctypes.c_double * max(1, n))(*sel_rows)
    od = (ctypes.c_uint32 * max(1, n))()
    if order is None:
        cost = ctypes.c_double(0)
        st = sel_star_plan_order(fact_rows, n, dr, sr, od, ctypes.byref(cost))
        if st != SEL_OK:
            raise SelError(st, "bad star plan input")
    else:
        for k, d in enumerate(order):
            od[k] = d
    inter = (ctypes.c_double * max(1, n))()
    c = float(sel_star_plan_cost(fact_rows, n, dr, sr, od, inter))
    if c < 0:
        raise SelError(SEL_E_INVALID, "bad star plan input")
    return [int(od[k]) for k in range(n)], c, [float(inter[k]) for k in range(n)]


class Context:
    """A libsel context bound to a device and a HIP stream (default: torch's
    current stream on that device)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.torch_stream = stream
        h = _vp()
        st = sel_ctx_create(device, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h))
        if st != SEL_OK:
            raise SelError(st, sel_last_error(None).decode())
        self.h = h
        self.device = device
        self._children = weakref.WeakSet()

    def close(self):
        """Destroy the context after every table and program made from it."""
        if self.h:
            kids = list(self._children)
            for kind in (Server, Batch, Program, DeviceTable):
                for k in kids:
                    if isinstance(k, kind):
                        k.destroy()
            sel_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return sel_last_error(self.h).decode()

    def check(self, st, ok=(SEL_OK,)):
        if st not in ok:
            raise SelError(st, self.error())
        return st

    @property
    def num_cus(self) -> int:
        return int(sel_ctx_num_cus(self.h))

    # ---- tables / programs
    def table(self, nrows: int, cols, keep=()):
        """cols: list of (type, dict_card, data_ptr, valid_ptr_or_None)."""
        return DeviceTable(self, nrows, cols, keep)

    def program(self, table, tree):
        return Program(self, table, tree)

    # ---- calls
    def count(self, table, prog) -> int:
        out = _u64(0)
        self.check(sel_count(self.h, table.h, prog.h, ctypes.byref(out)))
        return int(out.value)

    def count_async(self, table, prog, d_count_ptr: int):
        self.check(sel_count_async(self.h, table.h, prog.h, d_count_ptr))

    def pushdown_rowids(self, table, prog, max_rows: int, out_tensor, cap=None):
        """Returns (status, count); ids land in out_tensor[:count] on SEL_OK."""
        out = _u64(0)
        if cap is None:
            cap = 0 if out_tensor is None else out_tensor.numel()
        ptr = None if out_tensor is None else out_tensor.data_ptr()
        st = sel_pushdown_rowids(self.h, table.h, prog.h, max_rows, ptr, cap, ctypes.byref(out))
        self.check(st, ok=(SEL_OK, SEL_OVER_LIMIT, SEL_E_CAPACITY))
        return st, int(out.value)

    def pushdown_rowids_noalloc(self, table, prog, max_rows: int, out_tensor, cap=None):
        """pushdown_rowids over the library's fixed device workspace: the
        call allocates nothing.  Returns (status, count)."""
        out = _u64(0)
        if cap is None:
            cap = 0 if out_tensor is None else out_tensor.numel()
        ptr = None if out_tensor is None else out_tensor.data_ptr()
        st = sel_pushdown_rowids_noalloc(self.h, table.h, prog.h, max_rows, ptr, cap, ctypes.byref(out))
        self.check(st, ok=(SEL_OK, SEL_OVER_LIMIT, SEL_E_CAPACITY))
        return st, int(out.value)

    def factor_counts(self, table, prog):
        """(exact count, [exact count of each top-level AND factor]) in one
        batched launch; the factors in the program's evaluation order."""
        fc = (ctypes.c_uint64 * 32)()
        nf, cnt = _u32(0), _u64(0)
        self.check(sel_factor_counts(self.h, table.h, prog.h, 32, fc, ctypes.byref(nf), ctypes.byref(cnt)))
        return int(cnt.value), [int(fc[k]) for k in range(nf.value)]

    @staticmethod
    def independence_estimate(nrows: int, counts) -> float:
        arr = (ctypes.c_uint64 * max(1, len(counts)))(*counts)
        return float(sel_independence_estimate(nrows, len(counts), arr))

    def gather(self, table, ids_tensor, count: int, cols, outs, valid_outs=None):
        """Projected columns of a materialised selection: outs[c][:count] =
        column cols[c] at rows ids_tensor[:count]; valid_outs[c] (or None)
        receives the validity bits."""
        n = len(cols)
        cidx = (ctypes.c_uint32 * max(1, n))(*cols)
        optr = (ctypes.c_void_p * max(1, n))(*[o.data_ptr() for o in outs])
        vptr = None
        if valid_outs is not None:
            vptr = (ctypes.c_void_p * max(1, n))(*[v.data_ptr() if v is not None else None
                                                   for v in valid_outs])
        self.check(sel_gather(self.h, table.h, ids_tensor.data_ptr() if ids_tensor is not None else None,
                              count, n, cidx, optr, vptr))

    def select_pushdown(self, relations, min_table_size: int = 1000, max_selectivity: float = 0.05):
        """Algorithm 1 over [(table, program or None, out tensor or None)]:
        one dict per relation (decision, status, order, count, max_rows);
        the ids of a pushed relation land in its tensor[:count]."""
        n = len(relations)
        rels = (sel_spd_relation * max(1, n))()
        for i, (t, p, o) in enumerate(relations):
            rels[i].table = t.h
            rels[i].pred = p.h if p is not None else None
            rels[i].d_out = o.data_ptr() if o is not None else None
            rels[i].cap = o.numel() if o is not None else 0
        res = (sel_spd_result * max(1, n))()
        self.check(sel_select_pushdown(self.h, n, rels, min_table_size, max_selectivity, res))
        return [{"decision": SPD_DECISIONS[r.decision], "status": r.status,
                 "order": None if r.order == 0xFFFFFFFF else r.order,
                 "count": r.count, "max_rows": r.max_rows} for r in res[:n]]

    def pushdown_keybitmap(self, dim, key_col: int, key_min: int, prog, bitmap_tensor, nbits: int):
        """Returns (status, count); status SEL_OK or SEL_E_RANGE."""
        out = _u64(0)
        st = sel_pushdown_keybitmap(self.h, dim.h, key_col, key_min,
                                    prog.h if prog is not None else None,
                                    bitmap_tensor.data_ptr(), nbits, ctypes.byref(out))
        self.check(st, ok=(SEL_OK, SEL_E_RANGE))
        return st, int(out.value)

    def star_count(self, fact, fk_cols, bitmaps, nbits, fact_pred=None) -> int:
        n = len(fk_cols)
        fk = (_u32 * n)(*fk_cols)
        bm = (_vp * n)(*[b.data_ptr() for b in bitmaps])
        nb = (_u64 * n)(*nbits)
        out = _u64(0)
        self.check(sel_star_count(self.h, fact.h, fact_pred.h if fact_pred is not None else None,
                                  n, fk, bm, nb, ctypes.byref(out)))
        return int(out.value)

    def count_batch(self, pairs):
        """Exact counts of [(table, program), ...] in one launch."""
        n = len(pairs)
        ts = (_vp * n)(*[t.h.value for t, _ in pairs])
        ps = (_vp * n)(*[p.h.value for _, p in pairs])
        out = (_u64 * n)()
        self.check(sel_count_batch(self.h, n, ts, ps, out))
        return [int(x) for x in out]

    def batch(self, pairs):
        """A graph-captured batch (see Batch)."""
        return Batch(self, pairs)

    def autotune(self, table, prog, with_mask=False, reps=5):
        """Tune the scan's launch configuration for this program class and
        table size; returns (Launch, median ms)."""
        best, ms = sel_launch(), ctypes.c_double(0)
        self.check(sel_autotune(self.h, table.h, prog.h, 1 if with_mask else 0, reps,
                                ctypes.byref(best), ctypes.byref(ms)))
        return _launch(best), ms.value

    def autotune_batch(self, pairs, reps=3):
        n = len(pairs)
        ts = (_vp * n)(*[t.h.value for t, _ in pairs])
        ps = (_vp * n)(*[p.h.value for _, p in pairs])
        best, ms = sel_launch(), ctypes.c_double(0)
        self.check(sel_autotune_batch(self.h, n, ts, ps, reps, ctypes.byref(best), ctypes.byref(ms)))
        return _launch(best), ms.value

    def tune_save(self, path):
        self.check(sel_tune_save(self.h, str(path).encode()))

    def tune_load(self, path):
        self.check(sel_tune_load(self.h, str(path).encode()))

    @property
    def tune_entries(self) -> int:
        return int(sel_tune_entries(self.h))

    def star_program(self, fact, fk_cols, bitmaps, nbits, fact_pred=None):
        """The star semi-join as a program over the fact table (bitmaps are
        borrowed: keep the tensors alive while the program is used)."""
        return Program(self, fact, None, star=(fk_cols, bitmaps, nbits, fact_pred))

    def server(self, **cfg):
        return Server(self, **cfg)

    def set_launch(self, block=None, grid=0, cached=0, tiles_per_step=1, stage_words=0, rows_per_lane=0):
        if block is None:
            self.check(sel_ctx_set_launch(self.h, None))
        else:
            self.check(sel_ctx_set_launch(self.h, ctypes.byref(
                sel_launch(block, grid, cached, tiles_per_step, stage_words, rows_per_lane))))

    def enable_timing(self, on=True):
        self.check(sel_ctx_enable_timing(self.h, 1 if on else 0))

    def read_timing(self, reset=True):
        t = sel_timing()
        self.check(sel_ctx_read_timing(self.h, ctypes.byref(t), 1 if reset else 0))
        return [float(x) for x in t.ms], [int(x) for x in t.launches]


class Batch:
    """sel_batch: the batched count captured once in a HIP graph; run()
    replays it.  set_program(i, prog) swaps program i (same table) without a
    new capture."""

    def __init__(self, ctx: Context, pairs):
        self.ctx = ctx
        self.n = len(pairs)
        self._keep = list(pairs)
        ts = (_vp * self.n)(*[t.h.value for t, _ in pairs])
        ps = (_vp * self.n)(*[p.h.value for _, p in pairs])
        h = _vp()
        ctx.check(sel_batch_create(ctx.h, self.n, ts, ps, ctypes.byref(h)))
        self.h = h
        self._out = (_u64 * self.n)()
        ctx._children.add(self)

    def run(self):
        self.ctx.check(sel_batch_run(self.h, self._out))
        return [int(x) for x in self._out]

    def set_program(self, i: int, prog):
        self.ctx.check(sel_batch_set_program(self.h, i, prog.h))
        self._keep[i] = (self._keep[i][0], prog)

    def destroy(self):
        if getattr(self, "h", None):
            sel_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """sel_server: continuous batching of estimate requests over resident
    tables (cooperative scans, HBM-footprint admission, push-downs on their
    own stream)."""

    def __init__(self, ctx: Context, hbm_budget_bytes=0, chunk_rows=0, max_programs=0,
                 rounds_in_flight=0, rounds_per_cycle=0):
        self.ctx = ctx
        cfg = sel_server_config(hbm_budget_bytes, chunk_rows, max_programs, rounds_in_flight,
                                rounds_per_cycle, 0)
        h = _vp()
        ctx.check(sel_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self._pending = {}
        ctx._children.add(self)

    def submit(self, pairs, pushdown=None):
        """pairs: [(table, program), ...]; pushdown: None or (table, program,
        max_rows, out_tensor).  Returns a ticket."""
        n = len(pairs)
        ts = (_vp * max(1, n))(*[t.h.value for t, _ in pairs])
        ps = (_vp * max(1, n))(*[p.h.value for _, p in pairs])
        req = sel_request()
        req.nprog = n
        req.tables = ctypes.cast(ts, ctypes.POINTER(_vp))
        req.progs = ctypes.cast(ps, ctypes.POINTER(_vp))
        if pushdown is not None:
            pt, pp, mx, out = pushdown
            req.pd_table, req.pd_prog, req.pd_max_rows = pt.h.value, pp.h.value, mx
            req.pd_out, req.pd_cap = out.data_ptr(), out.numel()
        tk = _u64(0)
        self.ctx.check(sel_server_submit(self.h, ctypes.byref(req), ctypes.byref(tk)))
        self._pending[int(tk.value)] = (n, pairs, pushdown)
        return int(tk.value)

    def poll(self, ticket) -> bool:
        d = ctypes.c_int(0)
        self.ctx.check(sel_server_poll(self.h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def wait(self, ticket):
        """Returns (counts, pushdown status, pushdown count, latency ms)."""
        n, _, _ = self._pending.pop(ticket)
        counts = (_u64 * max(1, n))()
        res = sel_result()
        self.ctx.check(sel_server_wait(self.h, ticket, counts, ctypes.byref(res)))
        return [int(counts[i]) for i in range(n)], int(res.status), int(res.pd_count), res.latency_ms

    def stats(self, reset=False):
        st = sel_server_stats()
        self.ctx.check(sel_server_get_stats(self.h, ctypes.byref(st), 1 if reset else 0))
        return {k: getattr(st, k) for k, _ in sel_server_stats._fields_ if k != "pad"}

    def destroy(self):
        if getattr(self, "h", None):
            sel_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def max_rows(nrows: int, ratio: float) -> int:
    return int(sel_max_rows(nrows, ratio))


class DeviceTable:
    def __init__(self, ctx: Context, nrows: int, cols, keep=()):
        self.ctx = ctx
        self.nrows = nrows
        self._keep = list(keep)
        arr = _columns_struct(cols)
        h = _vp()
        ctx.check(sel_table_create(ctx.h, nrows, len(cols), arr, ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    def destroy(self):
        if getattr(self, "h", None):
            sel_table_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Program:
    def __init__(self, ctx: Context, table: DeviceTable, tree, star=None):
        self.ctx = ctx
        self.table = table
        h = _vp()
        if star is None:
            code, pool = flatten(tree)
            pbuf = ctypes.create_string_buffer(pool, max(1, len(pool)))
            ctx.check(sel_program_compile(ctx.h, table.h, code, len(code), pbuf, len(pool),
                                          ctypes.byref(h)))
        else:
            fk_cols, bitmaps, nbits, fact_pred = star
            n = len(fk_cols)
            self._bitmaps = list(bitmaps)
            ctx.check(sel_program_star(ctx.h, table.h, fact_pred.h if fact_pred is not None else None,
                                       n, (_u32 * n)(*fk_cols),
                                       (_vp * n)(*[b.data_ptr() for b in bitmaps]),
                                       (_u64 * n)(*nbits), ctypes.byref(h)))
        self.h = h
        ctx._children.add(self)

    @property
    def listing(self) -> str:
        return sel_program_listing(self.h).decode()

    @property
    def bytes_per_row(self) -> float:
        return float(sel_program_bytes_per_row(self.h))

    def destroy(self):
        if getattr(self, "h", None):
            sel_program_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def device_table(ctx: Context, host_table, device=None):
    """Copy a host table (objects with .columns of name/type/data/valid/
    dict_card numpy arrays) into device memory and describe it to libsel."""
    import torch
    dev = torch.device("cuda", ctx.device if device is None else device)
    cols, keep = [], []
    for c in host_table.columns:
        d = torch.from_numpy(np.ascontiguousarray(c.data)).to(dev)
        keep.append(d)
        vptr = None
        if c.valid is not None:
            v = torch.from_numpy(np.ascontiguousarray(c.valid).view(np.int32)).to(dev)
            keep.append(v)
            vptr = v.data_ptr()
        cols.append((c.type, c.dict_card, d.data_ptr(), vptr))
    torch.cuda.synchronize(dev)
    t = ctx.table(host_table.nrows, cols, keep)
    t.tensors = keep
    return t
