"""The learned gate end to end at reduced scale: exact labels from the
batched scan (checked against the oracle), featurization, GPU training,
held-out q-error, routing, and exactness of every routed predicate.

The q-error bound asserted here is statistical (parity unpinned): the
estimator is an approximation; what is pinned is that every count the gate
sends to exact evaluation equals the oracle's count."""
import numpy as np
import pytest

from oracle import features as fo
from oracle import scan
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc, learned

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def test_learned_gate_small(ctx):
    n = 4_000_000
    t = dg.table_learned(n, device="cuda")
    dt = esc.Table(t.nrows, t.dtypes, t.cols)
    host = t.host()
    cat = learned.Catalog.of(t, seed=2)
    specs = dg.preds_mixed(t, 16384 + 1024 + 2048, seed=dg.pred_seed(3))
    cps = [esc.Pred(dt, p) for p in specs]
    counts = learned.exact_counts(ctx, dt, cps)
    rng = np.random.default_rng(1)
    for i in rng.choice(len(specs), 150, replace=False):
        assert int(counts[i]) == scan.count(host, specs[i]), i
    est = learned.Estimator(ctx, dt, cat, dg.mlp_init(dg.MLP_SEED))
    x = est.features(cps)
    ocat = fo.Catalog(cat.cmin, cat.cmax, ["f" if d == dg.FLOAT32 else "i" for d in t.dtypes], cat.sample)
    assert np.array_equal(x[:50], fo.featurize_many(specs[:50], ocat))
    y = learned.labels(counts, n)
    tr, va, te = slice(0, 16384), slice(16384, 17408), slice(17408, None)
    loss, _ = est.train(x[tr], y[tr], epochs=20, batch=1024, lr=2e-3, order_seed=5)
    assert loss[-16:].mean() < 0.5 * loss[:16].mean()
    beta = learned.validation_beta(est.predict(x[va]), counts[va], n)
    yhat = est.predict(x[te])
    q = learned.q_error(learned.c_hat(yhat, n), counts[te], n)
    print("median q-error", float(np.median(q)), "beta", beta)
    assert np.median(q) < 2.5
    # routing, then exact evaluation of the routed predicates only
    route = esc.gate_pushdown(yhat, n, 0.05, beta, 1_000_000)
    want_route = np.array([fo.route_pushdown(float(v), n, 0.05, beta, 1_000_000) for v in yhat])
    assert np.array_equal(route, want_route)
    idx = np.flatnonzero(route) + te.start
    if len(idx):
        exact = learned.exact_counts(ctx, dt, [cps[i] for i in idx])
        for i, c in zip(idx[:100], exact[:100]):
            assert int(c) == scan.count(host, specs[i])
        assert np.array_equal(exact, counts[idx])
