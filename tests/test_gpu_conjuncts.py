"""Split selectivities (per-conjunct and prefix counts from one scan)
against the oracle's counts of the sub-predicates they are defined by."""
import numpy as np
import pytest

from oracle import scan
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def want_counts(t, spec):
    kids = spec[1] if spec[0] == "and" else [spec]
    conj = [scan.count(t, k) for k in kids]
    prefix = [scan.count(t, kids[0] if i == 0 else ("and", kids[:i + 1])) for i in range(len(kids))]
    return conj, prefix


@pytest.mark.parametrize("n", [0, 1, 1023, 4097, 20_001])
def test_random_trees(ctx, n):
    rng = np.random.default_rng(700 + n)
    cols = [rng.integers(-5, 6, n).astype(np.int32), rng.integers(0, 50, n).astype(np.int32),
            rng.choice(np.array([0.0, -0.0, 1.5, np.nan, np.inf], np.float32), n), rng.integers(0, 4, n).astype(np.int32)]
    t = dg.Table("tiny", n, [dg.INT32, dg.INT32, dg.FLOAT32, dg.DATE32], cols, ["u"] * 4, [None] * 4)
    dt = esc.device_table(t)
    done = 0
    for i in range(60):
        kids = [dg.random_pred_tiny(t, rng) for _ in range(int(rng.integers(1, 6)))]
        spec = ("and", kids) if len(kids) > 1 or rng.random() < 0.5 else kids[0]
        try:
            p = esc.Pred(dt, spec)
            got = ctx.count_conjuncts(dt, p)
        except esc.EscError as e:   # deep random trees may exceed the compiled limits
            assert e.status == esc.ERR_UNSUPPORTED
            continue
        assert got == want_counts(t, spec), (i, scan.to_sexpr(spec, t.dtypes))
        done += 1
    assert done >= 30


def test_star_conjunctions(ctx):
    t = dg.table_star(2_000_003, seed=95)
    dt = esc.device_table(t)
    for spec in dg.preds_star(t, 32, seed=96):
        p = esc.Pred(dt, spec)
        conj, prefix = ctx.count_conjuncts(dt, p)
        assert (conj, prefix) == want_counts(t, spec)
        assert prefix[-1] == ctx.count(dt, p)


def test_constant_conjuncts(ctx):
    t = dg.table_plain(10_000, seed=97)
    dt = esc.device_table(t)
    spec = ("and", [("lt", 1, 500), ("between", 2, -2**31, 2**31 - 1), ("lt", 0, -2**31), ("eq", 3, 7)])
    conj, prefix = ctx.count_conjuncts(dt, esc.Pred(dt, spec))
    assert conj[1] == t.nrows and conj[2] == 0
    assert prefix[2] == 0 and prefix[3] == 0
    assert (conj, prefix) == want_counts(t, spec)


def test_four_column_conjunction_repeatable(ctx):
    """A conjunction over four columns (float range, two small-domain IN-lists
    held as bitsets, a date range) counted ten times: identical and exact
    each time."""
    t = dg.table_star(2_000_003, seed=95)
    dt = esc.device_table(t)
    spec = ("and", [("lt", 4, np.float32(496.46582)), ("in", 2, [12, 46, 23, 24]), ("in", 3, [5, 3, 8, 9, 8]),
                    ("between", 1, 9304, 9421)])
    want = want_counts(t, spec)
    p = esc.Pred(dt, spec)
    for _ in range(10):
        assert ctx.count_conjuncts(dt, p) == want
