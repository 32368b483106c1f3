"""The library's featurization and gate (host code) against their CPU
oracle: features must match bit for bit, routing decisions exactly."""
import math

import numpy as np
import pytest

from oracle import features as fo
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc, learned


def _oracle_catalog(t, cat):
    return fo.Catalog(cat.cmin, cat.cmax, ["f" if d == dg.FLOAT32 else "i" for d in t.dtypes], cat.sample)


@pytest.mark.parametrize("rows", [0, 1, 7, 4096])
def test_featurize_matches_oracle_bitwise(rows):
    t = dg.table_mixed(50_000, 6, seed=3, kinds=dg.LEARNED_KINDS)
    cat = learned.Catalog.of(t, rows=rows, seed=rows) if rows else learned.Catalog.of(t, rows=1, seed=0)
    if not rows:
        cat.sample = None
    schema = esc.schema_table(t)
    preds = dg.preds_mixed(t, 200, seed=4) + dg.preds_anchored(t, 200, seed=5)
    cps = [esc.Pred(schema, p) for p in preds]
    got = esc.featurize(schema, cps, cat.cmin, cat.cmax, cat.sample)
    want = fo.featurize_many(preds, _oracle_catalog(t, cat))
    assert got.shape == want.shape == (400, 64)
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_featurize_golden_cases_through_library():
    from test_oracle_mlp import GOLDEN_DTYPES, GOLDEN_MAX, GOLDEN_MIN, _read_feature_golden, golden_sample
    schema = esc.Table(10, [dg.INT32, dg.INT32, dg.INT32, dg.INT32, dg.INT32, dg.FLOAT32])
    for case in _read_feature_golden():
        smp = golden_sample(case)
        got = esc.featurize(schema, [esc.Pred(schema, case["pred"])], GOLDEN_MIN, GOLDEN_MAX, smp)[0]
        want = fo.featurize(case["pred"], fo.Catalog(GOLDEN_MIN, GOLDEN_MAX, GOLDEN_DTYPES, smp))
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), case["pred"]


def test_featurize_errors():
    schema = esc.Table(10, [dg.INT32, dg.FLOAT32])
    p = esc.Pred(schema, ("eq", 0, 1))
    with pytest.raises(esc.EscError):
        esc.featurize(schema, [p], [5, np.float32(0)], [1, np.float32(1)])          # min above max
    with pytest.raises(esc.EscError):
        esc.featurize(schema, [p], [0, np.float32(np.nan)], [1, np.float32(1)])     # NaN bound
    with pytest.raises(ValueError):
        esc.featurize(schema, [p], [0, np.float32(0)], [1, np.float32(1)], [[0, 1], [0.5]])


def test_gate_matches_oracle():
    rng = np.random.default_rng(5)
    n = np.array([10**5, 10**6, 10**7, 10**8, 10**9])
    for tau, beta in [(0.05, 1.25), (0.05, 2.0), (0.2, 1.5), (1.0, 1.0)]:
        y = rng.uniform(-22, 1, 2000).astype(np.float32)
        nr = rng.choice(n, 2000)
        got = esc.gate_pushdown(y, nr, tau, beta, 10**6)
        want = np.array([fo.route_pushdown(float(a), int(b), tau, beta, 10**6) for a, b in zip(y, nr)])
        assert np.array_equal(got, want)
    for _ in range(500):
        yr, ys = (float(np.float32(v)) for v in rng.uniform(-15, 0, 2))
        nr, ns = (int(v) for v in rng.choice(n, 2))
        assert esc.gate_join_pair(yr, nr, ys, ns, 1.5) == fo.route_join_pair(yr, nr, ys, ns, 1.5)
    # a prediction exactly at tau is routed
    assert esc.gate_pushdown(np.array([math.log(0.05)], np.float32), 10**8, 0.05, 1.25, 10**6)[0]


def test_join_gate_with_ties_matches_oracle():
    rng = np.random.default_rng(6)
    for nr, ns, beta, tie in [(10**7, 10**8, 1.5, 1e-3), (10**7, 10**8, 1.5, 0.0), (10**6, 10**9, 2.0, 1e-2),
                              (10**8, 10**8, 1.25, 1e-5)]:
        yr = rng.uniform(-22, 1, 3000).astype(np.float32)
        ys = rng.uniform(-22, 1, 3000).astype(np.float32)
        got = esc.gate_join_pairs(yr, nr, ys, ns, beta, tie)
        want = np.array([fo.route_join_pair(float(a), nr, float(b), ns, beta, tie) for a, b in zip(yr, ys)])
        assert np.array_equal(got, want)
        assert 0 < got.sum() < len(got) or tie == 1e-2
    # ties only remove routes: routed with ties implies routed without
    yr = rng.uniform(-20, 0, 3000).astype(np.float32)
    ys = rng.uniform(-20, 0, 3000).astype(np.float32)
    with_tie = esc.gate_join_pairs(yr, 10**7, ys, 10**8, 1.5, 1e-3)
    without = esc.gate_join_pairs(yr, 10**7, ys, 10**8, 1.5, 0.0)
    assert not (with_tie & ~without).any() and (without & ~with_tie).any()
    assert len(esc.gate_join_pairs(np.zeros(0, np.float32), 10, np.zeros(0, np.float32), 10, 1.5, 0.0)) == 0
    with pytest.raises(esc.EscError):
        esc.gate_join_pairs(yr, 10**7, ys, 10**8, 1.5, 2.0)
    with pytest.raises(esc.EscError):
        esc.gate_join_pairs(yr, 0, ys, 10**8, 1.5, 0.0)


def test_catalog_handle_matches_featurize():
    """Features from a catalog built once equal esc_featurize's bit for bit."""
    from paper_1901_01488_amd import learned
    t = dg.tables_planning([50_000])[0]
    st = esc.Table(t.nrows, t.dtypes, None)
    cps = [esc.Pred(st, p) for p in dg.preds_mixed(t, 300, seed=3, min_conj=2, max_conj=6)]
    cat = learned.Catalog.of(t, seed=2)
    a = esc.featurize(st, cps, cat.cmin, cat.cmax, cat.sample)
    b = esc.Catalog(st, cat.cmin, cat.cmax, cat.sample).featurize(cps)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
