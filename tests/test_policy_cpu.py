"""Materialization policy: the oracle against hand-worked values and
invariants, and the library against the oracle (host code, no GPU)."""
import math

import numpy as np
import pytest

from oracle import policy as po
from paper_1901_01488_amd import esc

M0 = {"scan_bytes_per_s": 1e12, "fixed_s": 1e-5, "sparse_row_s": 1e-9, "dense_fraction": 0.01,
      "dense_bytes_per_s": 2e12, "dense_row_s": 1e-11, "tmp_bytes_per_s": 1e12}


def test_hand_worked_thresholds():
    # N = 1e8 rows, 3 columns re-read (12 bytes a row): T_scan = 1.2 ms.
    # Gathering regime: 1 ns + 12 bytes at 1e12 B/s = 1.012 ns a row; the
    # crossing (1.2 ms - 10 us) / 1.012 ns = 1.1759 % of the rows lies above
    # the dense fraction (1 %), so keeping pays through that regime.  Read
    # whole, the two projected columns cost 8e8 B / 2e12 B/s = 0.4 ms, and a
    # row 10 ps + 12 ps: crossing (1.19 ms - 0.4 ms) / 22 ps = 35.9 % of rows.
    tau, min_rows = po.thresholds(M0, 10**8, 3, 2, 1)
    assert math.isclose(tau, (1.19e-3 - 4e-4) / 2.2e-11 / 1e8, rel_tol=1e-12)
    assert math.isclose(tau, 0.35909090909090907, rel_tol=1e-12)
    assert math.isclose(min_rows, 1e-5 * 1e12 / 12, rel_tol=1e-12)   # N * 12 B / 1e12 B/s > 10 us
    # slower gathers: the crossing (1.19 ms / 10.012 ns = 0.11886 %) comes first
    m = dict(M0, sparse_row_s=1e-8)
    assert math.isclose(po.thresholds(m, 10**8, 3, 2, 1)[0], 1.19e-3 / 1.0012e-8 / 1e8, rel_tol=1e-12)
    # columns too slow to read whole (1.6 ms > the 1.19 ms left): keeping
    # stops where the write pass switches to whole columns
    m = dict(M0, dense_bytes_per_s=5e11)
    assert po.thresholds(m, 10**8, 3, 2, 1)[0] == 0.01
    # two reuses double the re-read and the temporary-table reads
    tau2, min2 = po.thresholds(M0, 10**8, 3, 2, 2)
    assert math.isclose(tau2, (2.4e-3 - 1e-5 - 4e-4) / (1e-11 + 2.4e-11) / 1e8, rel_tol=1e-12)
    assert math.isclose(min2, min_rows / 2, rel_tol=1e-12)
    # hand-worked costs of single selections (N = 1e8, k = 3, p = 2, r = 1)
    keep, saving = po.keep(M0, 10**8, 10**5, 3, 2, 1)        # s = 0.1 %: gathered
    assert keep and math.isclose(saving, 1.2e-3 - (1e-5 + 1e5 * 1e-9 + 1e5 * 1.2e-11), rel_tol=1e-12)
    keep, saving = po.keep(M0, 10**8, 5 * 10**7, 3, 2, 1)    # s = 50 %: columns read whole
    assert not keep and math.isclose(saving, 1.2e-3 - (1e-5 + 4e-4 + 5e7 * 2.2e-11), rel_tol=1e-12)


def test_free_materialization_reduces_to_byte_ratio():
    # no fixed or write cost and equal read rates: keep iff c (1 + p) < N k
    m = {"scan_bytes_per_s": 5e11, "fixed_s": 0.0, "sparse_row_s": 0.0, "dense_fraction": 1.0,
         "dense_bytes_per_s": 5e11, "dense_row_s": 0.0, "tmp_bytes_per_s": 5e11}
    n = 10**6
    for k, p in [(1, 0), (2, 1), (3, 2), (4, 1), (1, 3)]:
        tau, _ = po.thresholds(m, n, k, p, 1)
        assert math.isclose(tau, min(k / (1 + p), 1.0), rel_tol=1e-12)
        for c in [0, int(n * k / (1 + p)) - 1, int(n * k / (1 + p)) + 1, n]:
            if c <= n:
                assert po.keep(m, n, c, k, p, 1)[0] == (c * (1 + p) < n * k)


def _random_model(rng):
    return {"scan_bytes_per_s": 10 ** rng.uniform(11, 13), "fixed_s": float(rng.choice([0.0, 10 ** rng.uniform(-6, -3)])),
            "sparse_row_s": 10 ** rng.uniform(-11, -8), "dense_fraction": float(rng.choice([0.0, 1 / 128, 0.05, 1.0])),
            "dense_bytes_per_s": 10 ** rng.uniform(11, 13), "dense_row_s": 10 ** rng.uniform(-12, -9),
            "tmp_bytes_per_s": 10 ** rng.uniform(11, 13)}


def test_keep_agrees_with_thresholds():
    """keep holds for every selectivity below tau and not just above it;
    below min_rows even an empty result does not pay."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        m = _random_model(rng)
        n = int(10 ** rng.uniform(3, 9))
        k, p, r = int(rng.integers(1, 6)), int(rng.integers(0, 4)), int(rng.integers(1, 5))
        tau, min_rows = po.thresholds(m, n, k, p, r)
        assert 0.0 <= tau <= 1.0
        for c in np.unique(np.linspace(0, n, 257).astype(np.int64)):
            kept, saving = po.keep(m, n, int(c), k, p, r)
            assert kept == (saving > 0)
            if c < tau * n * (1 - 1e-9) and c > 0:
                assert kept, (m, n, k, p, r, tau, c)
        if tau < 1.0:
            above = int(math.ceil(tau * n * (1 + 1e-9))) + 1
            if above <= n:
                assert not po.keep(m, n, above, k, p, r)[0], (m, n, k, p, r, tau)
        assert po.keep(m, n, 0, k, p, r)[0] == (n > min_rows * (1 + 1e-12)) or \
            math.isclose(n, min_rows, rel_tol=1e-9)


def _model(d):
    return esc.CostModel(d["scan_bytes_per_s"], d["fixed_s"], d["sparse_row_s"], d["dense_fraction"],
                         d["dense_bytes_per_s"], d["dense_row_s"], d["tmp_bytes_per_s"])


def test_library_matches_oracle():
    rng = np.random.default_rng(4)
    for _ in range(150):
        d = _random_model(rng)
        n = int(10 ** rng.uniform(0, 9))
        k, p, r = int(rng.integers(1, 6)), int(rng.integers(0, 4)), int(rng.integers(1, 5))
        counts = np.unique(np.concatenate([[0, n], rng.integers(0, n + 1, 30),
                                           [int(n * d["dense_fraction"])]])).astype(np.uint64)
        counts = counts[counts <= n]
        keep, saving = esc.policy_keep(_model(d), n, counts, k, p, r)
        for c, kp, sv in zip(counts, keep, saving):
            want_k, want_s = po.keep(d, n, int(c), k, p, r)
            assert kp == want_k and sv == want_s
        assert esc.policy_thresholds(_model(d), n, k, p, r) == po.thresholds(d, n, k, p, r)


def test_library_errors():
    m = _model(M0)
    with pytest.raises(esc.EscError):
        esc.policy_keep(m, 10, [11], 2, 1)                       # count above nrows
    with pytest.raises(esc.EscError):
        esc.policy_keep(_model(dict(M0, scan_bytes_per_s=0.0)), 10, [1], 2, 1)
    with pytest.raises(esc.EscError):
        esc.policy_keep(_model(dict(M0, dense_fraction=1.5)), 10, [1], 2, 1)
    with pytest.raises(esc.EscError):
        esc.policy_keep(m, 10, [1], 0, 1)                        # nothing re-read
    with pytest.raises(esc.EscError):
        esc.policy_thresholds(m, 10, 2, 1, reuses=0)
