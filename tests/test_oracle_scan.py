"""Pins of the CPU scan oracle against facts that do not come from it.

- brute force by two independent evaluators written here (a pure-Python row
  loop and a numpy boolean-mask evaluator) on tiny and mid-size tables;
- closed forms on a permutation column (count(A < k) = k, ...);
- partition and inclusion-exclusion invariants;
- IEEE float32 and int32 edge cases with hand-derived counts;
- the hand-worked example of Section 1 (tests/golden/plain_example.txt);
- materialization invariants.
"""
import os

import numpy as np
import pytest

from oracle import scan
from paper_1901_01488_amd import datagen as dg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------- independent evaluators

def _wrap(x):
    return ((x + 2**31) % 2**32) - 2**31


def _py_expr(e, row):
    op = e[0]
    if op == "col":
        return int(row[e[1]])
    if op == "const":
        return int(e[1])
    a, b = _py_expr(e[1], row), _py_expr(e[2], row)
    if op == "add":
        return _wrap(a + b)
    if op == "sub":
        return _wrap(a - b)
    if op == "mul":
        return _wrap(a * b)
    if op == "mod":
        assert b > 0
        r = abs(a) % b
        return -r if a < 0 else r
    if op == "band":
        return _wrap(a & b)
    if op == "bor":
        return _wrap(a | b)
    if op == "bxor":
        return _wrap(a ^ b)
    if op == "shl":
        return _wrap(a << b)
    if op == "shr":
        return a >> b          # Python's >> on ints is the arithmetic shift
    raise ValueError(op)


def _py_test(t, v):
    if t[0] == "eq":
        return v == t[1]
    if t[0] == "lt":
        return v < t[1]
    if t[0] == "gt":
        return v > t[1]
    if t[0] == "between":
        return t[1] <= v <= t[2]
    return any(v == k for k in t[1])


def py_eval(p, row, dtypes):
    """Pure-Python truth value of predicate p on one row (floats compared as
    Python floats: float32 -> float64 is exact, so IEEE order is kept)."""
    op = p[0]
    if op == "and":
        return all(py_eval(q, row, dtypes) for q in p[1])
    if op == "or":
        return any(py_eval(q, row, dtypes) for q in p[1])
    if op == "udf":
        return _py_test(p[2], _py_expr(p[1], row))
    v = row[p[1]]
    v = float(v) if dtypes[p[1]] == dg.FLOAT32 else int(v)
    conv = (lambda k: float(k)) if dtypes[p[1]] == dg.FLOAT32 else int
    if op == "in":
        return _py_test(("in", [conv(k) for k in p[2]]), v)
    return _py_test((op,) + tuple(conv(k) for k in p[2:]), v)


def np_mask(p, cols, dtypes):
    """numpy boolean-mask evaluation (vectorised, int64 arithmetic for udfs)."""
    op = p[0]
    if op == "and":
        m = np.ones(len(cols[0]), bool)
        for q in p[1]:
            m &= np_mask(q, cols, dtypes)
        return m
    if op == "or":
        m = np.zeros(len(cols[0]), bool)
        for q in p[1]:
            m |= np_mask(q, cols, dtypes)
        return m
    if op == "udf":
        v = _np_expr(p[1], cols)
        return _np_test(p[2][0], v, [np.int64(k) for k in (p[2][1] if p[2][0] == "in" else p[2][1:])])
    v = cols[p[1]]
    if dtypes[p[1]] == dg.FLOAT32:
        ks = [np.float32(k) for k in (p[2] if op == "in" else p[2:])]
    else:
        v = v.astype(np.int64)
        ks = [np.int64(k) for k in (p[2] if op == "in" else p[2:])]
    return _np_test(op, v, ks)


def _np_test(op, v, ks):
    if op == "eq":
        return v == ks[0]
    if op == "lt":
        return v < ks[0]
    if op == "gt":
        return v > ks[0]
    if op == "between":
        return (v >= ks[0]) & (v <= ks[1])
    m = np.zeros(len(v), bool)
    for k in ks:
        m |= v == k
    return m


def _np_expr(e, cols):
    if e[0] == "col":
        return cols[e[1]].astype(np.int64)
    if e[0] == "const":
        return np.full(len(cols[0]), e[1], np.int64)
    a, b = _np_expr(e[1], cols), _np_expr(e[2], cols)
    w = lambda x: ((x + 2**31) % 2**32) - 2**31
    op = e[0]
    if op == "add":
        return w(a + b)
    if op == "sub":
        return w(a - b)
    if op == "mul":
        return w((a * b) & 0xFFFFFFFF)
    if op == "mod":
        return np.fmod(a, b)                  # C-style truncated remainder
    if op == "band":
        return a & b
    if op == "bor":
        return a | b
    if op == "bxor":
        return a ^ b
    if op == "shl":
        return w((a << b) & 0xFFFFFFFF)
    if op == "shr":
        return a >> b
    raise ValueError(op)


# ----------------------------------------------------------- brute force

def _tiny_table(rng, n):
    cols = [rng.integers(-5, 6, n).astype(np.int32),
            rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32),
            rng.choice(np.array([0.0, -0.0, 1.0, -1.0, 2.5, np.inf, -np.inf, np.nan, 1e-45, -1e-45],
                                np.float32), n),
            rng.integers(0, 4, n).astype(np.int32)]
    return dg.Table("tiny", n, [dg.INT32, dg.INT32, dg.FLOAT32, dg.DATE32], cols,
                    ["u", "u", "f", "u"], [None] * 4)


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 17, 64])
def test_brute_force_tiny(n):
    rng = np.random.default_rng(100 + n)
    t = _tiny_table(rng, n)
    rows = list(zip(*[c.tolist() for c in t.cols])) if n else []
    for _ in range(150):
        p = dg.random_pred_tiny(t, rng)
        want = np.array([py_eval(p, r, t.dtypes) for r in rows], bool)
        got = scan.eval_rows(t, p)
        assert np.array_equal(got, want), scan.to_sexpr(p, t.dtypes)
        assert scan.count(t, p) == int(want.sum())
        if n:
            assert np.array_equal(np_mask(p, t.cols, t.dtypes), want)


def test_brute_force_mid_numpy():
    t = dg.table_mixed(100_000, 6, seed=5, kinds=dg.LEARNED_KINDS)
    preds = dg.preds_mixed(t, 40, seed=6)
    for p in preds:
        want = np_mask(p, t.cols, t.dtypes)
        assert scan.count(t, p) == int(want.sum())


def test_brute_force_plain_config_small():
    t = dg.table_plain(20_000, seed=11)
    rows = list(zip(*[c.tolist() for c in t.cols]))
    for s in range(5):
        p = dg.pred_plain(t, s)
        want = np.array([py_eval(p, r, t.dtypes) for r in rows], bool)
        assert scan.count(t, p) == int(want.sum())
        assert np.array_equal(np_mask(p, t.cols, t.dtypes), want)


def test_brute_force_star_small():
    t = dg.table_star(50_000, seed=12)
    for p in dg.preds_star(t, 32, seed=13):
        assert scan.count(t, p) == int(np_mask(p, t.cols, t.dtypes).sum())


# ----------------------------------------------------------- closed forms

@pytest.fixture(scope="module")
def perm_table():
    return dg.table_plain(100_000, seed=21)


def test_closed_forms_permutation(perm_table):
    t = perm_table
    n = t.nrows
    for k in [0, 1, 2, 999, 50_000, n - 1, n, n + 5]:
        assert scan.count(t, ("lt", 0, k)) == min(k, n)
    for k in [-1, 0, 7, n - 2, n - 1]:
        assert scan.count(t, ("gt", 0, k)) == n - 1 - k
    for k in [0, 1, 12345, n - 1]:
        assert scan.count(t, ("eq", 0, k)) == 1
    assert scan.count(t, ("eq", 0, n)) == 0
    for a, b in [(0, 0), (5, 10), (0, n - 1), (100, 99), (n - 3, n + 10)]:
        want = max(0, min(b, n - 1) - max(a, 0) + 1)
        assert scan.count(t, ("between", 0, a, b)) == want
    s = [3, 3, 7, 99_999, 100_000, -1, 55]
    assert scan.count(t, ("in", 0, s)) == len({v for v in s if 0 <= v < n})
    assert scan.count(t, ("gt", 0, -2**31)) == n
    assert scan.count(t, ("lt", 0, -2**31)) == 0


def test_partitions(perm_table):
    t = perm_table
    n = t.nrows
    assert sum(scan.count(t, ("eq", 1, x)) for x in range(1000)) == n
    udf = dg.UDF_PLAIN
    assert sum(scan.count(t, ("udf", udf, ("eq", w))) for w in range(97)) == n
    for k in [0, 17, 500, 999, -3, 1000]:
        parts = [scan.count(t, (op, 1, k)) for op in ("lt", "eq", "gt")]
        assert sum(parts) == n


def test_inclusion_exclusion(perm_table):
    t = perm_table
    rng = np.random.default_rng(31)
    small = dg.table_mixed(30_000, 6, seed=32, kinds=dg.LEARNED_KINDS)
    for tab in (t, small):
        for _ in range(20):
            p = dg.random_pred_tiny(tab, rng)
            q = dg.random_pred_tiny(tab, rng)
            cp, cq = scan.count(tab, p), scan.count(tab, q)
            cand = scan.count(tab, ("and", [p, q]))
            cor = scan.count(tab, ("or", [p, q]))
            assert cor == cp + cq - cand
            assert cand <= min(cp, cq)


def test_between_is_difference_of_lt(perm_table):
    t = perm_table
    for a, b in [(0, 10), (100, 500), (3, 3), (0, 999)]:
        assert scan.count(t, ("between", 1, a, b)) == scan.count(t, ("lt", 1, b + 1)) - scan.count(t, ("lt", 1, a))


# ----------------------------------------------------------- IEEE and int32 edges

EDGE_CASES = [
    (("eq", 0, 0.0), 2), (("eq", 0, -0.0), 2), (("lt", 0, 0.0), 5), (("gt", 0, 0.0), 7),
    (("lt", 0, np.nan), 0), (("gt", 0, np.nan), 0), (("eq", 0, np.nan), 0),
    (("between", 0, -np.inf, np.inf), 14), (("between", 0, 1e-45, 1.17549435e-38), 3),
    (("gt", 0, 1e-45), 6), (("lt", 0, -1e-45), 4), (("eq", 0, 1e-45), 1),
    (("in", 0, [0.0, np.nan, 1.0]), 3), (("between", 0, 0.0, -0.0), 2),
    (("lt", 0, -np.inf), 0), (("gt", 0, np.inf), 0), (("lt", 0, np.inf), 13),
    (("between", 0, 1.0, -1.0), 0), (("between", 0, np.nan, 1.0), 0),
    (("lt", 1, -2**31), 0), (("gt", 1, 2**31 - 1), 0), (("between", 1, -2**31, 2**31 - 1), 16),
    (("eq", 1, 5), 3), (("lt", 1, 0), 6), (("gt", 1, 2**31 - 2), 1), (("between", 1, 5, 4), 0),
    (("in", 1, [5, 5, 7]), 4),
    (("udf", ("add", ("col", 1), ("const", 1)), ("gt", 0)), 9),
    (("udf", ("mod", ("col", 1), ("const", 7)), ("eq", 0)), 4),
    (("udf", ("mod", ("col", 1), ("const", 7)), ("lt", 0)), 5),
    (("udf", ("shr", ("col", 1), ("const", 31)), ("eq", -1)), 6),
]


def edge_pred(pred, t):
    """EDGE_CASES entries with float32 constants on the float column."""
    if pred[0] == "udf" or t.dtypes[pred[1]] != dg.FLOAT32:
        return pred
    if pred[0] == "in":
        return ("in", pred[1], [np.float32(v) for v in pred[2]])
    return (pred[0], pred[1]) + tuple(np.float32(v) for v in pred[2:])


@pytest.mark.parametrize("pred,want", EDGE_CASES)
def test_edge_values(pred, want):
    t = dg.table_edge_floats()
    assert scan.count(t, edge_pred(pred, t)) == want


# ----------------------------------------------------------- golden example

def _read_golden():
    rows, cases = [], []
    with open(os.path.join(GOLDEN, "plain_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#") or line.startswith("table"):
                continue
            if line.startswith("case"):
                kv = dict(tok.split("=") for tok in line.split()[1:])
                cases.append({k: [int(x) for x in v.split(",")] for k, v in kv.items()})
            else:
                rows.append([int(x) for x in line.split()])
    return np.array(rows, np.int32), cases


def test_golden_section1_example():
    data, cases = _read_golden()
    t = dg.Table("R", len(data), [dg.INT32] * 4, [data[:, j].copy() for j in range(4)])
    for case in cases:
        p = ("and", [("eq", 1, 3), ("between", 2, 100, 250), ("or", [("eq", 3, 7), ("gt", 3, 50)]),
                     ("udf", dg.UDF_PLAIN, ("gt", case["w"][0]))])
        c, ids, (a, cc, d) = scan.materialize(t, p, dg.PLAIN_PROJECTION)
        assert c == case["count"][0]
        assert ids.tolist() == case["rowids"]
        assert a.tolist() == case["A"] and cc.tolist() == case["C"] and d.tolist() == case["D"]


# ----------------------------------------------------------- materialize invariants

def test_materialize_invariants():
    t = dg.table_star(40_000, seed=41)
    for p in dg.preds_star(t, 8, seed=42):
        c, ids, outs = scan.materialize(t, p, dg.STAR_PROJECTION)
        assert c == scan.count(t, p) == len(ids)
        assert np.all(np.diff(ids) > 0)
        mask = np_mask(p, t.cols, t.dtypes)
        assert np.array_equal(np.flatnonzero(mask), ids)
        for j, o in zip(dg.STAR_PROJECTION, outs):
            assert np.array_equal(o.view(np.uint32), t.cols[j][ids].view(np.uint32))


def test_materialize_everything_and_capacity():
    t = dg.table_plain(5_000, seed=43)
    c, ids, (a,) = scan.materialize(t, ("gt", 0, -1), [0])
    assert c == t.nrows and np.array_equal(ids, np.arange(t.nrows))
    assert np.array_equal(a, t.cols[0])
    c, ids, _ = scan.materialize(t, ("lt", 0, 100), [1], capacity=99)
    assert c == 100 and len(ids) == 99 and np.array_equal(ids, np.flatnonzero(t.cols[0] < 100)[:99])


def test_oracle_rejects_bad_input():
    d = [dg.INT32, dg.FLOAT32]
    assert scan.check(d, "(eq 0 5)")
    assert not scan.check(d, "(eq 1 5)")              # float column needs a float constant
    assert not scan.check(d, "(eq 0 fx3f800000)")     # int column given a float constant
    assert not scan.check(d, "(eq 2 5)")              # no such column
    assert not scan.check(d, "(in 0)")                # empty IN
    assert not scan.check(d, "(and)")
    assert not scan.check(d, "(udf (col 1) (gt 0))")  # float column in a udf
    assert not scan.check(d, "(eq 0 5")
    assert not scan.check(d, "(eq 0 99999999999)")
