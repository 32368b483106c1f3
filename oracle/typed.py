"""Oracle for predicates on TEXT and DECIMAL columns (Section 3, Table 3).

TEST INFRASTRUCTURE ONLY: used by the tests, never by the product path.

Evaluates a predicate on the columns' own values, with no encoding: a TEXT
column is a sequence of Python strings compared as strings (code-point
order, which for UTF-8 is the byte-wise order), a DECIMAL column a sequence
of decimal.Decimal values compared exactly with Decimal(literal).  Integer
and float columns are compared as numbers.  Leaves: ("eq"|"lt"|"gt", c, v),
("between", c, a, b) inclusive on both ends, ("in", c, [v...]) and
("prefix", c, s) on TEXT columns; inner nodes ("and"|"or", [children]).
"""
from __future__ import annotations

from decimal import Decimal

import numpy as np


def _key(v, kind):
    return Decimal(str(v)) if kind == "decimal" else v


def _leaf(col, kind, leaf):
    op = leaf[0]
    if op == "prefix":
        p = leaf[2]
        return np.fromiter((x.startswith(p) for x in col), dtype=bool, count=len(col))
    if op == "in":
        ks = {_key(v, kind) for v in leaf[2]}
        return np.fromiter((x in ks for x in col), dtype=bool, count=len(col))
    a = _key(leaf[2], kind)
    if op == "eq":
        f = lambda x: x == a
    elif op == "lt":
        f = lambda x: x < a
    elif op == "gt":
        f = lambda x: x > a
    elif op == "between":
        b = _key(leaf[3], kind)
        f = lambda x: a <= x <= b
    else:
        raise ValueError(op)
    return np.fromiter((f(x) for x in col), dtype=bool, count=len(col))


def eval_rows(cols, kinds, pred) -> np.ndarray:
    """Qualifying-row mask; kinds[c] in {"int", "text", "decimal"}."""
    op = pred[0]
    if op in ("and", "or"):
        masks = [eval_rows(cols, kinds, q) for q in pred[1]]
        out = masks[0].copy()
        for m in masks[1:]:
            out = (out & m) if op == "and" else (out | m)
        return out
    return _leaf(cols[pred[1]], kinds[pred[1]], pred)


def count(cols, kinds, pred) -> int:
    return int(eval_rows(cols, kinds, pred).sum())
