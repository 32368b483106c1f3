"""Learned gate in front of exact selectivity computation.

Exact selectivity computation runs a COUNT(*) sub-query per selection
(Section 2).  The gate asks a small learned estimator first and keeps the
exact count for the predicates whose estimate lies close enough to a plan
decision that the estimator's error could flip it: the push-down /
materialization threshold on selectivity (Section 2.1) and the order in which
build relations are joined (Section 2.2).  The estimator is trained on exact
counts produced by the batched scan, so exact ESC is both its teacher and its
fallback.

This module sequences library calls (scan, featurization, MLP, gate); every
count, feature, forward, backward and update runs inside libesc.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import esc


def exact_counts(ctx, table: esc.Table, preds, group=1024):
    """Exact counts of many compiled predicates over one table, by the
    batched kernel in groups of at most `group` predicates per pass."""
    out = np.zeros(len(preds), np.uint64)
    step = 16384
    for i in range(0, len(preds), step):
        chunk = preds[i:i + step]
        b = esc.Batch(ctx, [table], chunk, [0] * len(chunk), group=group)
        out[i:i + len(chunk)] = b.count()
        del b
    return out


def labels(counts, n):
    """y = ln(max(c, 1) / n)."""
    return np.log(np.maximum(np.asarray(counts, np.float64), 1.0) / float(n)).astype(np.float32)


def q_error(c_hat, c, n):
    c_hat = np.clip(np.asarray(c_hat, np.float64), 1.0, float(n))
    cp = np.maximum(np.asarray(c, np.float64), 1.0)
    return np.maximum(c_hat / cp, cp / c_hat)


def c_hat(yhat, n):
    return np.clip(float(n) * np.exp(np.asarray(yhat, np.float64)), 1.0, float(n))


class Catalog:
    """Column statistics the featurization reads: minimum, maximum and a
    uniform row sample (the same rows for every column) of the first six
    columns, as host values."""

    SAMPLE_ROWS = 4096

    def __init__(self, cmin, cmax, sample=None):
        self.cmin, self.cmax, self.sample = list(cmin), list(cmax), sample

    @classmethod
    def of(cls, table, rows=SAMPLE_ROWS, seed=0):
        """From a datagen table whose columns are numpy arrays or device
        tensors."""
        cols = table.cols
        n = table.nrows
        idx = np.random.default_rng(seed).integers(0, max(n, 1), rows if n else 0)
        if cols and not isinstance(cols[0], np.ndarray):   # device tensors
            import torch
            ti = torch.from_numpy(idx).to(cols[0].device)
            cmin = [c.min().item() for c in cols]
            cmax = [c.max().item() for c in cols]
            sample = [c[ti].cpu().numpy() for c in cols[:6]]
        else:
            cmin = [c.min() for c in cols]
            cmax = [c.max() for c in cols]
            sample = [np.asarray(c)[idx] for c in cols[:6]]
        return cls(cmin, cmax, sample if n else None)


class Estimator:
    """Featurization + MLP for one table."""

    def __init__(self, ctx, schema: esc.Table, catalog: Catalog, params):
        self.ctx, self.schema, self.catalog = ctx, schema, catalog
        self.mlp = esc.MLP(ctx, params)
        self.nrows = schema.nrows

    def features(self, preds):
        if getattr(self, "_lib_catalog", None) is None:
            c = self.catalog
            self._lib_catalog = esc.Catalog(self.schema, c.cmin, c.cmax, c.sample)
        return self._lib_catalog.featurize(preds)

    def train(self, x, y, epochs, batch, lr, order_seed):
        import torch
        from . import datagen as dg
        n = x.shape[0]
        order = dg.minibatch_order(n, batch, epochs, order_seed)
        dev = f"cuda:{self.ctx.device}"
        xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        yt = torch.from_numpy(np.ascontiguousarray(y, np.float32)).to(dev)
        ot = torch.from_numpy(order).to(dev)
        t0 = time.perf_counter()
        loss = self.mlp.train(xt, yt, ot, len(order) // batch, batch, lr=lr)
        return loss, time.perf_counter() - t0

    def fit(self, x, y, phases, batch, order_seed):
        """Training in phases of (epochs, learning rate), Adam state carried
        over (a step-wise decaying schedule); returns (loss of the last
        phase, seconds)."""
        total = 0.0
        loss = None
        for i, (epochs, lr) in enumerate(phases):
            loss, s = self.train(x, y, epochs=epochs, batch=batch, lr=lr, order_seed=order_seed + i)
            total += s
        return loss, total

    def predict(self, x):
        import torch
        dev = f"cuda:{self.ctx.device}"
        xt = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
        return self.mlp.predict(xt).cpu().numpy()


def validation_beta(yhat, counts, n, quantile=0.95, floor=1.25):
    """Band factor: the 95th-percentile validation q-error, at least 1.25."""
    q = q_error(c_hat(yhat, n), counts, n)
    return max(floor, float(np.quantile(q, quantile)))
