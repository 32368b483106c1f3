"""Planning workload at reduced scale: arriving three-table queries decided
plain (one count per selection), batched (one graph launch per micro-batch)
and batched with the learned gate.  Every exact count must agree with the
plain path; the gate's gain over the method without it is measured."""
import numpy as np
import pytest

from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc, learned, planning

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def test_planning_gate_gain(ctx):
    sizes = [2_000_000, 20_000_000, 200_000_000]
    tabs = dg.tables_planning(sizes, device="cuda")
    dts = [esc.Table(t.nrows, t.dtypes, t.cols) for t in tabs]
    nq = 300
    qs = [dg.preds_mixed(t, nq, seed=dg.pred_seed(4) + i, min_conj=2, max_conj=6) for i, t in enumerate(tabs)]
    queries = list(zip(*qs))
    arrivals = dg.poisson_arrivals(nq, 5000.0, seed=4)
    # one estimator per table, trained offline on exact labels
    ests = []
    for i, (t, dt) in enumerate(zip(tabs, dts)):
        specs = dg.preds_mixed(t, 8192, seed=dg.pred_seed(4) + 100 + i, min_conj=2, max_conj=6)
        cps = [esc.Pred(dt, p) for p in specs]
        cnt = learned.exact_counts(ctx, dt, cps)
        e = learned.Estimator(ctx, dt, learned.Catalog.of(t, seed=9 + i), dg.mlp_init(dg.MLP_SEED))
        x = e.features(cps)
        e.train(x, learned.labels(cnt, t.nrows), epochs=15, batch=1024, lr=2e-3, order_seed=9 + i)
        ests.append(e)
    w = planning.Workload(ctx, dts, queries, arrivals)
    plain = w.run_plain()
    batched = w.run_batched()
    assert np.array_equal(batched["counts"], plain["counts"])
    g = planning.GateConfig(beta=1.5)
    gated = w.run_batched(gate=True, estimators=ests, gcfg=g)
    r = gated["routed"]
    assert np.array_equal(gated["counts"][r], plain["counts"][r])
    print({k: v for k, v in plain.items() if k != "counts"})
    print({k: v for k, v in batched.items() if k != "counts"})
    print({k: v for k, v in gated.items() if k not in ("counts", "est", "routed")})
    # the probe relation (largest) is never scanned with the gate on
    assert not r[:, 2].any()
    assert gated["predicates_per_s"] > batched["predicates_per_s"]
    assert gated["predicates_per_s"] > plain["predicates_per_s"]
