"""Input generators: properties the workloads rely on (CPU only)."""
import numpy as np

from oracle import scan
from paper_1901_01488_amd import datagen as dg


def test_anchored_predicates_select_their_row():
    t = dg.table_learned(20_000, seed=3)
    h = t.host()
    specs = dg.preds_anchored(t, 200, seed=4)
    counts = np.array([scan.count(h, p) for p in specs])
    assert counts.min() >= 1
    # selectivities spread over several decades
    sel = counts / t.nrows
    assert sel.min() < 1e-3 and sel.max() > 0.3
