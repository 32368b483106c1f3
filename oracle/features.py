"""CPU oracle of the 64-dimensional predicate featurization and of the gate.

TEST INFRASTRUCTURE ONLY: used by tests and the smoke check, never by the
product path.

Featurization (the learned estimator's input; the paper has no estimator,
so this is the build's definition).  For each of the first six columns c,
ten float32 values at offset 10*c:

  [present, lo, hi, is_eq, is_lt, is_gt, is_between, is_in, in_size/16, in_or]

  present     1 if some leaf references column c
  lo, hi      the constraint the conjunction puts on c, normalised to [0,1]
              with the catalog minimum and maximum (0 and 1 when free)
  is_*        1 if some leaf on c uses that comparison
  in_size     total length of the IN-lists on c, divided by 16
  in_or       1 if some leaf on c sits under an OR

followed by four global values [n_conj/6, n_or/6, has_udf, n_leaves/16].

Normalisation of a constant v of column c, every step rounded to float32:
  d = f32(v) - f32(min_c); s = f32(max_c) - f32(min_c); q = d / s,
  clamped to [0, 1]; 0 when s == 0 or v is NaN.
Leaf intervals: eq k -> [k,k]; lt k -> [min, k]; gt k -> [k, max];
between a b -> [a, b]; in S -> [min S, max S].  A conjunct that is a leaf
intersects its interval into its column's [lo, hi]; a conjunct that is an
OR of leaves on one column intersects the union hull of their intervals;
anything else only sets flags.  Conjuncts are the children of a root AND,
or the root itself.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 64
NCOLF = 6
F32 = np.float32


def _norm(v, lo, hi):
    v, lo, hi = F32(v), F32(lo), F32(hi)
    if np.isnan(v):
        return F32(0.0)
    s = F32(hi - lo)
    if s == 0 or np.isnan(s):
        return F32(0.0)
    q = F32(F32(v - lo) / s)
    return F32(min(max(q, F32(0.0)), F32(1.0)))


def _leaf_interval(leaf, cmin, cmax):
    op, c = leaf[0], leaf[1]
    n = lambda v: _norm(v, cmin[c], cmax[c])
    if op == "eq":
        return n(leaf[2]), n(leaf[2])
    if op == "lt":
        return F32(0.0), n(leaf[2])
    if op == "gt":
        return n(leaf[2]), F32(1.0)
    if op == "between":
        return n(leaf[2]), n(leaf[3])
    vals = [F32(v) if not isinstance(v, (int, np.integer)) else v for v in leaf[2]]
    return n(min(vals)), n(max(vals))


def featurize(pred, cmin, cmax):
    f = np.zeros(NFEAT, np.float32)
    for c in range(NCOLF):
        f[10 * c + 2] = 1.0
    counts = {"leaves": 0, "or": 0, "udf": 0}
    opslot = {"eq": 3, "lt": 4, "gt": 5, "between": 6, "in": 7}

    def flags(p, under_or):
        op = p[0]
        if op in ("and", "or"):
            if op == "or":
                counts["or"] += 1
            for q in p[1]:
                flags(q, under_or or op == "or")
            return
        counts["leaves"] += 1
        if op == "udf":
            counts["udf"] = 1
            return
        c = p[1]
        if c >= NCOLF:
            return
        f[10 * c] = 1.0
        f[10 * c + opslot[op]] = 1.0
        if op == "in":
            f[10 * c + 8] = F32(f[10 * c + 8] + F32(len(p[2])) / F32(16.0))
        if under_or:
            f[10 * c + 9] = 1.0

    def clamp(c, lo, hi):
        if c >= NCOLF:
            return
        f[10 * c + 1] = max(f[10 * c + 1], lo)
        f[10 * c + 2] = min(f[10 * c + 2], hi)

    flags(pred, False)
    conj = pred[1] if pred[0] == "and" else [pred]
    for q in conj:
        if q[0] in ("eq", "lt", "gt", "between", "in"):
            lo, hi = _leaf_interval(q, cmin, cmax)
            clamp(q[1], lo, hi)
        elif q[0] == "or" and all(k[0] in ("eq", "lt", "gt", "between", "in") for k in q[1]) \
                and len({k[1] for k in q[1]}) == 1:
            iv = [_leaf_interval(k, cmin, cmax) for k in q[1]]
            clamp(q[1][0][1], min(a for a, _ in iv), max(b for _, b in iv))
    f[60] = F32(len(conj)) / F32(6.0)
    f[61] = F32(counts["or"]) / F32(6.0)
    f[62] = F32(counts["udf"])
    f[63] = F32(counts["leaves"]) / F32(16.0)
    return f


def featurize_many(preds, cmin, cmax):
    return np.stack([featurize(p, cmin, cmax) for p in preds]) if preds else np.zeros((0, NFEAT), np.float32)


# ------------------------------------------------------------------ gate

def log_sel(yhat, n):
    """Predicted ln-selectivity clamped to [ln(1/n), 0] (i.e. c_hat in [1, n])."""
    return min(max(float(yhat), -math.log(float(n))), 0.0)


def route_pushdown(yhat, n, tau, beta, min_rows):
    """Exact evaluation is worth it when the push-down decision (selectivity
    below tau, on a table larger than min_rows; Section 2.1) could flip
    within the estimator's error factor beta: tau/beta <= s_hat <= tau*beta."""
    if n < min_rows:
        return False
    s = log_sel(yhat, n)
    return math.log(tau) - math.log(beta) <= s <= math.log(tau) + math.log(beta)


def route_join_pair(yhat_r, n_r, yhat_s, n_s, beta):
    """The build-side join order (smallest filtered relation first; Section
    2.2) could flip when 1/beta^2 <= c_hat_R / c_hat_S <= beta^2."""
    lr = log_sel(yhat_r, n_r) + math.log(float(n_r))
    ls = log_sel(yhat_s, n_s) + math.log(float(n_s))
    d = lr - ls
    return -2.0 * math.log(beta) <= d <= 2.0 * math.log(beta)
