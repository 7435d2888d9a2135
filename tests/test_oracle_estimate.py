"""CPU pins of the oracle's conjunct counts and the independence estimate
(Ch.1 sec.1.1): the thesis' worked numbers, a grid on which independence
holds exactly, and a conjunct repeated, where it fails by a known factor."""
import os

import numpy as np

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_example.txt")


def golden():
    vals = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        vals[k] = float(v)
    return vals


def test_paper_worked_example():
    g = golden()
    n = int(g["relation_rows_R"])
    sels = [g["sel_R_A_eq_x"], g["sel_R_B_lt_y1"], g["sel_R_B_gt_y2"], g["sel_R_C_or"]]
    est = oracle.independence_estimate(n, [s * n for s in sels])
    # the product the thesis prints, to its four decimals, and the rows it implies
    assert round(est / n, 4) == g["independence_product"]
    assert round(n * g["independence_product"]) == g["estimated_rows"]
    # the true selection, and how far the plan it would pick is off
    assert round(n * g["true_selectivity"]) == g["true_rows"]
    assert round(g["true_rows"] / g["relation_rows_S"]) == g["plan_ratio"]
    # the estimate is two orders of magnitude low: 100.2M / 903,612
    q = oracle.q_error(est, g["true_rows"])
    assert 110.8 < q < 111.0


def grid_table(n=10_000):
    r = np.arange(n)
    t = datagen.Table("grid", n)
    t.columns.append(datagen.Column("a", "i32", (r % 100).astype(np.int32)))
    t.columns.append(datagen.Column("b", "i32", (r // 100).astype(np.int32)))
    t.columns.append(datagen.Column("id", "i32", r.astype(np.int32)))
    return t


def test_independent_grid_is_exact():
    # a = r mod 100 and b = r div 100 take every pair once: a < 10 and b < 20
    # hold together on 10 x 20 rows, and the product estimate is exact
    t = grid_table()
    tree = ("and", ("cmp", 0, "<", 10), ("cmp", 1, "<", 20))
    c, fc = oracle.factor_counts(t, tree)
    assert (c, fc) == (200, [1000, 2000])
    assert oracle.independence_estimate(t.nrows, fc) == 200.0
    assert oracle.q_error(200.0, c) == 1.0


def test_repeated_conjunct_and_flattening():
    # the same test twice (exact: its 1000 rows; independence: 10000 * 0.1 *
    # 0.1 = 100) and an OR
    t = grid_table()
    leaf = ("cmp", 2, "<", 1000)
    tree = ("and", leaf, ("and", leaf, ("or", ("cmp", 0, "=", 3), ("cmp", 1, "=", 3))))
    assert oracle.and_factors(tree) == [leaf, leaf, tree[2][2]]
    c, fc = oracle.factor_counts(t, tree)
    # the OR holds on a = 3 (100 rows) or b = 3 (100 rows), 199 rows; with
    # id < 1000 (b < 10): a = 3 on 10 rows, b = 3 on 100 rows, both on 1
    assert fc == [1000, 1000, 199] and c == 109
    # estimate 10000 * 0.1 * 0.1 * 0.0199 = 1.99 rows against 109
    est = oracle.independence_estimate(t.nrows, fc)
    assert abs(est - 1.99) < 1e-9
    assert abs(oracle.q_error(est, c) - 109 / 1.99) < 1e-6
    assert oracle.and_factors(("or", leaf, leaf)) == [("or", leaf, leaf)]
    assert oracle.q_error(0, 0) == 1.0


def test_join_formula_on_the_worked_example():
    """Ch.1 sec.1.1: with the estimated |sigma(R)| the plan (sigma(R) join S)
    join T looks cheapest (0.9 M against the 5 M of S join T); with the true
    count its first join holds 100.2 M rows, 20 times the other plan's."""
    g = golden()
    R, S, T = g["relation_rows_R"], g["relation_rows_S"], g["relation_rows_T"]
    # S.A and T.B are primary keys: V(S, A) = |S|, V(T, B) = |T|, and the
    # referencing sides hold at most that many distinct values
    est_first = oracle.join_size(g["estimated_rows"], S, S, S)
    other_first = oracle.join_size(S, T, T, T)
    assert est_first == 900_000 and other_first == 5_000_000
    true_first = oracle.join_size(g["true_rows"], S, S, S)
    assert true_first == 100_200_000
    assert round(true_first / other_first) == g["plan_ratio"]
    assert R > S > T


def test_star_plan_by_hand():
    # fractions 0.5, 0.1, 0.3 of 1000, 100, 10 keys; 1e6 fact rows: the
    # cheapest order keeps the smallest fractions first
    dims, sels = [1000, 100, 10], [500, 10, 3]
    order, cost = oracle.best_star_plan(1e6, dims, sels)
    assert order == [1, 2, 0]
    c, inter = oracle.star_plan_cost(1e6, dims, sels, order)
    assert inter == [1e5, 3e4, 1.5e4] and c == cost == 1.45e5
    assert oracle.star_plan_cost(1e6, dims, sels, [0, 2, 1])[0] == 5e5 + 1.5e5 + 1.5e4
