"""The C-ABI library loads and exports every symbol include/sel.h declares;
the host-side program compiler validates and lowers programs (no GPU)."""
import os
import re

import numpy as np
import pytest

from paper_1806_08384_amd import sel

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(sel_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(sel._lib, n)]
    assert not missing, missing
    # and the binding wraps each of them
    assert not [n for n in names if n not in sel.EXPORTED], [n for n in names if n not in sel.EXPORTED]


def test_max_rows():
    assert sel.max_rows(1000, 0.0) == 0
    assert sel.max_rows(1000, 1.0) == 1000
    assert sel.max_rows(1000, 0.0441) == 44
    assert sel.max_rows(75_000_000, 0.044) == 3_300_000
    assert sel.max_rows(10, 2.0) == 10
    assert sel.max_rows(10, -1.0) == 0
    assert sel.max_rows(2 ** 32 - 1, 0.5) == (2 ** 32 - 1) // 2


I32 = ("i32", 0, False)
I32N = ("i32", 0, True)
I8 = ("i8", 0, False)
I64N = ("i64", 0, True)
D25 = ("i32", 25, True)


def lowered(tree, cols=(I32, I32N, I8, I64N, D25)):
    st, text, err = sel.check_program(100, list(cols), tree)
    assert st == sel.SEL_OK, err
    return text.strip().splitlines()


def test_lowering_comparisons():
    assert lowered(("cmp", 0, "<", 3000)) == ["RANGE i32 lo=-2147483648 hi=2999"]
    assert lowered(("cmp", 0, ">=", 7000)) == ["RANGE i32 lo=7000 hi=2147483647"]
    assert lowered(("cmp", 0, ">", 5)) == ["RANGE i32 lo=6 hi=2147483647"]
    assert lowered(("cmp", 0, "<=", 5)) == ["RANGE i32 lo=-2147483648 hi=5"]
    assert lowered(("cmp", 0, "=", 5)) == ["RANGE i32 lo=5 hi=5"]
    assert lowered(("cmp", 0, "<>", 5)) == ["RANGE i32 lo=5 hi=5", "NOT"]
    assert lowered(("between", 1, 3500, 6499)) == ["RANGE i32 lo=3500 hi=6499 nullable"]


def test_lowering_out_of_type_literals():
    # int8 column: literals beyond the type fold to constants (no NULLs)
    assert lowered(("cmp", 2, "<", 300)) == ["TRUE"]
    assert lowered(("cmp", 2, ">", 300)) == ["FALSE"]
    assert lowered(("cmp", 2, "=", -129)) == ["FALSE"]
    assert lowered(("cmp", 2, ">=", -128)) == ["TRUE"]
    # on a nullable column they keep NULL rows UNKNOWN
    assert lowered(("cmp", 1, "<", sel.INT64_MIN)) == ["NONNULL_FALSE"]
    assert lowered(("cmp", 3, ">", sel.INT64_MAX)) == ["NONNULL_FALSE"]
    assert lowered(("cmp", 3, ">=", sel.INT64_MIN)) == ["NONNULL_TRUE"]
    assert lowered(("between", 1, 10, 5)) == ["NONNULL_FALSE"]
    assert lowered(("cmp", 1, "<>", 2 ** 40)) == ["NONNULL_FALSE", "NOT"]


def test_lowering_in_lists():
    assert lowered(("in", 0, (7,))) == ["RANGE i32 lo=7 hi=7"]
    assert lowered(("in", 0, (3, 4, 5, 4, 3))) == ["RANGE i32 lo=3 hi=5"]
    assert lowered(("in", 0, tuple(range(0, 20, 2)))) == ["BITMAP i32 base=0 nbits=19"]
    assert lowered(("in", 0, (-5, 10 ** 6))) == ["INLIST i32 n=2 hashed"]
    # a list longer than the hashed limit keeps only its sorted form
    assert lowered(("in", 0, tuple(range(0, 100_000 * 1025, 100_000)))) == ["INLIST i32 n=1025"]
    assert lowered(("in", 2, (1000, 2000))) == ["FALSE"]           # no int8 value
    assert lowered(("in", 1, (2 ** 40,))) == ["NONNULL_FALSE"]


def test_lowering_merges_ranges_of_a_column():
    """Range tests of one column under one conjunction become the test of
    the ranges' intersection (exact in three-valued logic); tests under an
    OR, or on other columns, stay apart."""
    assert lowered(("and", ("between", 0, 0, 1999), ("cmp", 2, "<", 45), ("cmp", 0, ">=", 10))) == [
        "RANGE i32 lo=10 hi=1999", "RANGE i8 lo=-128 hi=44 guard_and", "AND"]
    assert lowered(("and", ("cmp", 1, ">", 5), ("and", ("cmp", 1, "<", 9), ("cmp", 1, "<>", 7)))) == [
        "RANGE i32 lo=6 hi=8 nullable", "RANGE i32 lo=7 hi=7 nullable", "NOT", "AND"]
    # disjoint ranges: FALSE on non-NULL rows, UNKNOWN on NULL ones
    assert lowered(("and", ("cmp", 1, "<", 5), ("cmp", 1, ">", 9))) == ["NONNULL_FALSE"]
    assert lowered(("and", ("cmp", 0, "<", 5), ("cmp", 0, ">", 9))) == ["FALSE"]
    assert lowered(("or", ("cmp", 0, "<", 5), ("cmp", 0, ">", 9))) == [
        "RANGE i32 lo=-2147483648 hi=4", "RANGE i32 lo=10 hi=2147483647 guard_or", "OR"]


def test_lowering_codesets_and_nulls():
    words = np.zeros(1, dtype=np.uint32)
    # a LIKE matching no dictionary code: empty code set, NULL rows stay UNKNOWN
    assert lowered(("codeset", 4, 25, words)) == ["NONNULL_FALSE"]
    words[0] = 0b1010
    assert lowered(("codeset", 4, 25, words)) == ["BITMAP i32 base=0 nbits=25 nullable"]
    assert lowered(("isnull", 0)) == ["FALSE"]
    assert lowered(("notnull", 0)) == ["TRUE"]
    assert lowered(("isnull", 1)) == ["ISNULL"]


def test_guards_and_reordering():
    t = ("and", ("cmp", 0, "<", 5), ("codeset", 4, 25, np.array([6], dtype=np.uint32)))
    assert lowered(t) == ["RANGE i32 lo=-2147483648 hi=4",
                          "BITMAP i32 base=0 nbits=25 nullable guard_and", "AND"]
    # a leaf AND a deeper subtree: the subtree is evaluated first
    t = ("and", ("cmp", 0, "<", 5), ("or", ("cmp", 1, "=", 1), ("cmp", 1, "=", 2)))
    assert lowered(t) == ["RANGE i32 lo=1 hi=1 nullable", "RANGE i32 lo=2 hi=2 nullable guard_or",
                          "OR", "RANGE i32 lo=-2147483648 hi=4 guard_and", "AND"]


def test_deep_programs_fit_after_reordering():
    # a right-deep chain of 20 ANDs needs depth 21 as written, 2 after reordering
    t = ("cmp", 0, "=", 0)
    for k in range(1, 21):
        t = ("and", ("cmp", 0, "=", k), t)
    code, pool = sel.flatten(t)
    assert len(code) == 41
    lowered(t)


def check_err(tree_or_code, cols=(I32, I32N, I8, I64N, D25), pool=b""):
    colst = sel._columns_struct([(ty, card, None, 8 if n else None) for ty, card, n in cols])
    if isinstance(tree_or_code, tuple):
        code, pool = sel.flatten(tree_or_code)
    else:
        code = tree_or_code
    return sel.check_raw(100, colst, code, pool)


def raw(*instrs):
    arr = (sel.sel_instr * len(instrs))()
    for i, (op, col, aux, a, b) in enumerate(instrs):
        arr[i].op, arr[i].col, arr[i].aux, arr[i].a, arr[i].b = op, col, aux, a, b
    return arr


def test_validation_errors():
    OP = sel.OP
    st, _, err = check_err(raw((OP["="], 9, 0, 1, 0)))
    assert st == sel.SEL_E_INVALID and "column" in err
    st, _, err = check_err(raw((OP["="], 0, 0, 1, 0), (OP["and"], 0, 0, 0, 0)))
    assert st == sel.SEL_E_INVALID and "underflow" in err
    st, _, err = check_err(raw((OP["="], 0, 0, 1, 0), (OP["="], 0, 0, 2, 0)))
    assert st == sel.SEL_E_INVALID and "stack" in err
    st, _, err = check_err(raw((99, 0, 0, 0, 0)))
    assert st == sel.SEL_E_INVALID and "unknown op" in err
    st, _, err = check_err(raw((OP["in"], 0, 0, 0, 2)), pool=b"\0" * 8)
    assert st == sel.SEL_E_INVALID and "out of bounds" in err
    st, _, err = check_err(raw((OP["in"], 0, 4, 0, 1)), pool=b"\0" * 16)
    assert st == sel.SEL_E_INVALID and "misaligned" in err
    st, _, err = check_err(raw((OP["in"], 0, 0, 0, 0)), pool=b"\0" * 8)
    assert st == sel.SEL_E_INVALID
    st, _, err = check_err(raw((OP["codeset"], 0, 0, 0, 10)), pool=b"\0" * 8)
    assert st == sel.SEL_E_TYPE
    st, _, err = check_err(raw((OP["codeset"], 4, 0, 0, 100)), pool=b"\0" * 8)
    assert st == sel.SEL_E_INVALID
    st, _, err = check_err(raw(*[(OP["true"], 0, 0, 0, 0)] * 65))
    assert st == sel.SEL_E_INVALID and "length" in err
    st, _, err = check_err(raw())
    assert st == sel.SEL_E_INVALID
    # a balanced tree of 32 leaves needs depth 6: fine; depth 9 cannot be reached in 64 instrs
    leaves = [("cmp", 0, "=", k) for k in range(32)]
    while len(leaves) > 1:
        leaves = [("or", leaves[i], leaves[i + 1]) for i in range(0, len(leaves), 2)]
    st, text, err = check_err(leaves[0])
    assert st == sel.SEL_OK, err
    with pytest.raises(ValueError):
        sel.flatten(("cmp", 0, "<", 2 ** 63))
