"""CPU oracle of the 64-dimensional predicate featurization and of the gate.

TEST INFRASTRUCTURE ONLY: used by tests and the smoke check, never by the
product path.

Featurization (the learned estimator's input; the paper has no estimator,
so this is the build's definition).  For each of the first six columns c,
ten float32 values at offset 10*c:

  [lsel, lo, hi, is_eq, is_lt, is_gt, is_between, in_mass, in_size/16, in_or]

followed by four global values [n_conj/6, n_or/6, has_udf, n_leaves/16].
Everything is computed in float64 and rounded to float32 once at the end.

Column CDF.  From the catalog minimum and maximum of the column and a row
sample (values that are NaN or outside [min, max] are dropped; m = number
kept), with u_1 < ... < u_k the distinct sampled values:
  knot u_j carries a left limit  L_j = (#{s < u_j} + 1/2) / m
                and a right limit R_j = (#{s <= u_j} - 1/2) / m;
  a knot (min, 0, 0) goes in front unless min == u_1, in which case L_1 = 0;
  a knot (max, 1, 1) goes behind unless max == u_k, in which case R_k = 1;
  G(v) = 0 below the first knot, 1 above the last, L_j / R_j at a knot
  (for "below v" / "at most v"), and between knots a and b the straight line
  from R_a to L_b.
F_below(v) and F_atmost(v) are G(v) with the left / right limit for a
float32 column; an integer column (int32, date32) uses G(v - 1/2) and
G(v + 1/2).  A NaN constant maps to 0.  With no sample, the knots are just
(min, 0, 0) and (max, 1, 1): the CDF of a uniform column.

Leaf ranges [a, b]: eq k -> [F_below(k), F_atmost(k)]; lt k -> [0, F_below(k)];
gt k -> [F_atmost(k), 1]; between x y -> [F_below(x), F_atmost(y)];
in S -> [F_below(min S), F_atmost(max S)] over the non-NaN constants
([0, 0] if there are none).

Per column (leaves at any depth): is_eq / is_lt / is_gt / is_between are 1
if some leaf on the column uses that comparison; every IN leaf adds its
number of constants / 16 to in_size and, to in_mass, the sum over its
distinct non-NaN constants v (ascending) of F_atmost(v) - F_below(v).
The conjuncts are the children of a root AND, or the root itself; the j-th
conjunct (1-based) that contains an OR marks every leaf inside it with j/4,
and in_or is the largest mark of the column's leaves.

lo / hi start at 0 / 1 and are intersected with: the range of each leaf
conjunct; for an OR conjunct whose children are all leaves, the hull (min a,
max b) of its leaves on each column -- for every column if the OR has one
column, else only for columns that no leaf conjunct constrains.

lsel: 0 for a column no leaf mentions; otherwise with est = max(hi - lo, 0),
replaced by in_mass when in_size > 0, in_mass > 0 and in_mass < est,
lsel = min((0 - ln(max(est, 1e-9))) / 20.72326583694641, 1) (0 - x, not -x,
so that an unconstrained column gives +0).

Globals: conjunct count / 6, number of OR nodes / 6, 1 if any udf leaf,
number of leaves / 16.
"""
from __future__ import annotations

import math

import numpy as np

NFEAT = 64
NCOLF = 6
LEAVES = ("eq", "lt", "gt", "between", "in")


class ColumnCdf:
    """The smoothed sample CDF of one column (see the module docstring)."""

    def __init__(self, lo, hi, is_int, sample=()):
        lo, hi = float(lo), float(hi)
        vals = sorted(float(v) for v in sample if not math.isnan(float(v)) and lo <= float(v) <= hi)
        m = len(vals)
        knots = []   # [value, left limit, right limit]
        i = 0
        while i < m:
            j = i
            while j < m and vals[j] == vals[i]:
                j += 1
            knots.append([vals[i], (i + 0.5) / m, (j - 0.5) / m])
            i = j
        if not knots or lo < knots[0][0]:
            knots.insert(0, [lo, 0.0, 0.0])
        else:
            knots[0][1] = 0.0
        if hi > knots[-1][0]:
            knots.append([hi, 1.0, 1.0])
        else:
            knots[-1][2] = 1.0
        self.knots = knots
        self.is_int = is_int

    def _g(self, v, atmost):
        k = self.knots
        if v < k[0][0]:
            return 0.0
        if v > k[-1][0]:
            return 1.0
        for idx, (u, left, right) in enumerate(k):
            if u == v:
                return right if atmost else left
            if u > v:
                pu, _, pright = k[idx - 1]
                t = (v - pu) / (u - pu)
                return pright + t * (left - pright)
        raise AssertionError

    def below(self, v):
        v = float(v)
        if math.isnan(v):
            return 0.0
        return self._g(v - 0.5, False) if self.is_int else self._g(v, False)

    def atmost(self, v):
        v = float(v)
        if math.isnan(v):
            return 0.0
        return self._g(v + 0.5, True) if self.is_int else self._g(v, True)


class Catalog:
    """Per-column CDFs for the first six columns.  dtypes: 'i' for int32 /
    date32, 'f' for float32; sample: per column a list of values, or None."""

    def __init__(self, cmin, cmax, dtypes, sample=None):
        n = min(len(dtypes), NCOLF)
        self.cdf = [ColumnCdf(cmin[c], cmax[c], dtypes[c] != "f", () if sample is None else sample[c])
                    for c in range(n)]


def _values(leaf):
    return sorted(set(float(v) for v in leaf[2] if not math.isnan(float(v))))


def _range(leaf, cat):
    op, c = leaf[0], leaf[1]
    F = cat.cdf[c]
    if op == "eq":
        return F.below(leaf[2]), F.atmost(leaf[2])
    if op == "lt":
        return 0.0, F.below(leaf[2])
    if op == "gt":
        return F.atmost(leaf[2]), 1.0
    if op == "between":
        return F.below(leaf[2]), F.atmost(leaf[3])
    vals = _values(leaf)
    if not vals:
        return 0.0, 0.0
    return F.below(vals[0]), F.atmost(vals[-1])


def _has_or(p):
    if p[0] == "or":
        return True
    return p[0] == "and" and any(_has_or(q) for q in p[1])


def featurize(pred, cat):
    f = [0.0] * NFEAT
    for c in range(NCOLF):
        f[10 * c + 2] = 1.0
    present = [False] * NCOLF
    stats = {"leaves": 0, "or": 0, "udf": 0}
    opslot = {"eq": 3, "lt": 4, "gt": 5, "between": 6}

    def visit(p, mark):
        if p[0] in ("and", "or"):
            if p[0] == "or":
                stats["or"] += 1
            for q in p[1]:
                visit(q, mark)
            return
        stats["leaves"] += 1
        if p[0] == "udf":
            stats["udf"] = 1
            return
        c = p[1]
        if c >= NCOLF:
            return
        present[c] = True
        if p[0] == "in":
            F = cat.cdf[c]
            mass = 0.0
            for v in _values(p):
                mass += F.atmost(v) - F.below(v)
            f[10 * c + 7] += mass
            f[10 * c + 8] += len(p[2]) / 16.0
        else:
            f[10 * c + opslot[p[0]]] = 1.0
        f[10 * c + 9] = max(f[10 * c + 9], mark)

    conj = pred[1] if pred[0] == "and" else [pred]
    j = 0
    for q in conj:
        mark = 0.0
        if _has_or(q):
            j += 1
            mark = j / 4.0
        visit(q, mark)

    def narrow(c, a, b):
        f[10 * c + 1] = max(f[10 * c + 1], a)
        f[10 * c + 2] = min(f[10 * c + 2], b)

    bound_by_leaf = {q[1] for q in conj if q[0] in LEAVES}
    for q in conj:
        if q[0] in LEAVES:
            if q[1] < NCOLF:
                narrow(q[1], *_range(q, cat))
        elif q[0] == "or" and all(k[0] in LEAVES for k in q[1]):
            cols = []
            for k in q[1]:
                if k[1] not in cols:
                    cols.append(k[1])
            for c in cols:
                if c >= NCOLF or (len(cols) > 1 and c in bound_by_leaf):
                    continue
                rs = [_range(k, cat) for k in q[1] if k[1] == c]
                narrow(c, min(a for a, _ in rs), max(b for _, b in rs))
    for c in range(NCOLF):
        if not present[c]:
            continue
        est = max(f[10 * c + 2] - f[10 * c + 1], 0.0)
        if f[10 * c + 8] > 0.0 and 0.0 < f[10 * c + 7] < est:
            est = f[10 * c + 7]
        f[10 * c] = min((0.0 - math.log(max(est, 1e-9))) / 20.72326583694641, 1.0)
    f[60] = len(conj) / 6.0
    f[61] = stats["or"] / 6.0
    f[62] = float(stats["udf"])
    f[63] = stats["leaves"] / 16.0
    return np.array(f, dtype=np.float32)


def featurize_many(preds, cat):
    return np.stack([featurize(p, cat) for p in preds]) if preds else np.zeros((0, NFEAT), np.float32)


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


def route_join_pair(yhat_r, n_r, yhat_s, n_s, beta, tie_sel=0.0):
    """The build-side join order (smallest filtered relation first; Section
    2.2) could flip when 1/beta^2 <= c_hat_R / c_hat_S <= beta^2.

    Ties: the relation probed first passes sel * |P| of the probe
    relation's rows on to the second lookup (Section 2.2 probes the largest
    relation against the others' hash tables), so when both selectivities,
    even multiplied by beta, are at most tie_sel, the orders differ by at
    most tie_sel * |P| lookups and neither needs an exact count.  tie_sel =
    0 turns ties off."""
    sr, ss = log_sel(yhat_r, n_r), log_sel(yhat_s, n_s)
    if tie_sel > 0.0:
        top = math.log(tie_sel) - math.log(beta)
        if sr <= top and ss <= top:
            return False
    d = (sr + math.log(float(n_r))) - (ss + math.log(float(n_s)))
    return -2.0 * math.log(beta) <= d <= 2.0 * math.log(beta)
