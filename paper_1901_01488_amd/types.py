"""TEXT and DECIMAL predicate columns, lowered onto their 4-byte storage.

Section 3 (Table 3) measures predicates on TEXT and DECIMAL(15,2) columns.
Here a TEXT column is stored as dictionary codes (rank in the dictionary's
byte-wise order) and a DECIMAL(p, s) column as value * 10^s in int32, or,
when its values exceed int32, in int64 held as two 32-bit word columns
(split_words); the library translates a string or decimal comparison into a code range or an
exact int32 bound (esc_dict_range, esc_decimal_bound), and `lower` rewrites
a predicate description into int32 leaves on the stored values, which the
ordinary compiler and kernels then evaluate.  Everything here runs on the
host; the library's dictionary and decimal routines do the comparisons.

Extra leaf forms on typed columns: ("eq"|"lt"|"gt", c, v), ("between", c,
a, b), ("in", c, [v...]) with str constants on TEXT columns and decimal
literals (str or decimal.Decimal) on DECIMAL columns, and ("prefix", c, s)
on TEXT columns.
"""
from __future__ import annotations

import ctypes
from decimal import Decimal

import numpy as np

from . import esc

I32_MIN, I32_MAX = -2**31, 2**31 - 1


def _c_str(s):
    """UTF-8 bytes of s for a NUL-terminated C string (NUL is refused)."""
    if "\x00" in s:
        raise ValueError("TEXT values and literals may not contain NUL: %r" % s)
    return s.encode()


class Dict:
    """An esc_dict over distinct strings (UTF-8; the byte-wise order is the
    code-point order)."""

    def __init__(self, strings):
        strs = [_c_str(s) for s in strings]
        arr = (ctypes.c_char_p * max(len(strs), 1))(*strs)
        h = ctypes.c_void_p()
        esc.check(esc.lib().esc_dict_create(arr, len(strs), ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int()
        esc.check(esc.lib().esc_dict_size(self.h, ctypes.byref(n)))
        out = ctypes.c_char_p()
        self.strings = []
        for c in range(n.value):
            esc.check(esc.lib().esc_dict_string(self.h, c, ctypes.byref(out)))
            self.strings.append(out.value.decode())

    def encode(self, values):
        """int32 codes of a sequence of strings; each must be in the
        dictionary (KeyError names the first one that is not)."""
        idx = {s: i for i, s in enumerate(self.strings)}
        try:
            return np.fromiter((idx[v] for v in values), dtype=np.int32, count=len(values))
        except KeyError as e:
            raise KeyError(f"{e.args[0]!r} is not in the dictionary") from None

    def range(self, op, s, s2=None):
        """Code interval (lo, hi) of esc_dict_range; (0, -1) when empty."""
        lo, hi = ctypes.c_int32(), ctypes.c_int32()
        esc.check(esc.lib().esc_dict_range(self.h, op, _c_str(s), _c_str(s2) if s2 is not None else None,
                                           ctypes.byref(lo), ctypes.byref(hi)))
        return lo.value, hi.value

    def __del__(self):
        if getattr(self, "h", None) and esc._lib is not None:
            esc._lib.esc_dict_destroy(self.h)
            self.h = None


def decimal_bound(literal, scale, op):
    """(bound, empty) of esc_decimal_bound for a literal given as a string
    or a decimal.Decimal (written out in positional notation)."""
    text = format(literal, "f") if isinstance(literal, Decimal) else str(literal)
    b, e = ctypes.c_int64(), ctypes.c_int()
    esc.check(esc.lib().esc_decimal_bound(text.encode(), int(scale), op, ctypes.byref(b), ctypes.byref(e)))
    return b.value, bool(e.value)


def _range_leaf(c, lo, hi):
    """lo <= x <= hi on int32 column c (int64 bounds; empty -> false)."""
    lo, hi = max(lo, I32_MIN), min(hi, I32_MAX)
    if lo > hi:
        return ("lt", c, I32_MIN)
    return ("between", c, int(lo), int(hi))


def _text_leaf(d: Dict, leaf):
    op, c = leaf[0], leaf[1]
    if op == "in":
        codes = sorted({lo for lo, hi in (d.range(esc.EQ, v) for v in leaf[2]) if lo <= hi})
        return ("in", c, codes) if codes else ("lt", c, I32_MIN)
    if op == "prefix":
        return _range_leaf(c, *d.range(esc.DICT_PREFIX, leaf[2]))
    if op == "between":
        return _range_leaf(c, *d.range(esc.BETWEEN, leaf[2], leaf[3]))
    return _range_leaf(c, *d.range({"eq": esc.EQ, "lt": esc.LT, "gt": esc.GT}[op], leaf[2]))


def _decimal_leaf(scale, leaf):
    op, c = leaf[0], leaf[1]
    if op == "in":
        vals = sorted({v for v, e in (decimal_bound(x, scale, esc.EQ) for x in leaf[2]) if not e})
        vals = [v for v in vals if I32_MIN <= v <= I32_MAX]
        return ("in", c, vals) if vals else ("lt", c, I32_MIN)
    if op == "eq":
        v, empty = decimal_bound(leaf[2], scale, esc.EQ)
        return ("lt", c, I32_MIN) if empty else _range_leaf(c, v, v)
    if op == "lt":
        return _range_leaf(c, I32_MIN, decimal_bound(leaf[2], scale, esc.LT)[0])
    if op == "gt":
        return _range_leaf(c, decimal_bound(leaf[2], scale, esc.GT)[0], I32_MAX)
    if op == "between":   # a <= x <= b: above the largest value below a, below the smallest above b
        lo = decimal_bound(leaf[2], scale, esc.LT)[0] + 1
        hi = decimal_bound(leaf[3], scale, esc.GT)[0] - 1
        return _range_leaf(c, lo, hi)
    raise ValueError(f"{op} is not a decimal comparison")


# ---------------------------------------------------------------- 64-bit decimals as two word columns
#
# A DECIMAL(15,2) value needs up to 10^15 stored units, beyond int32.  Such
# a column is stored as two 4-byte columns: H = the high 32 bits (signed)
# and L = the low 32 bits with the sign bit flipped, so that the signed
# order of L is the unsigned order of the low word.  The order of the 64-bit
# values is then the lexicographic order of (H, L), and every comparison
# with a 64-bit bound becomes a few int32 leaves on H and L; the scans keep
# their 16-byte loads and 32-bit compares and read 8 bytes per row.

def split_words(x):
    """(H, L) int32 word columns of an int64 array (numpy or torch)."""
    if isinstance(x, np.ndarray):
        x = x.astype(np.int64)
        hi = (x >> 32).astype(np.int32)
        lo = ((x & 0xFFFFFFFF) ^ 0x80000000).astype(np.uint32).view(np.int32)
        return hi, lo
    import torch
    hi = (x >> 32).to(torch.int32)
    lo = ((x & 0xFFFFFFFF) ^ 0x80000000)
    lo = torch.where(lo >= 2**31, lo - 2**32, lo).to(torch.int32)
    return hi, lo


def _words(c):
    h = c >> 32
    lo = (c & 0xFFFFFFFF) ^ 0x80000000
    return h, lo - 2**32 if lo >= 2**31 else lo


def _range64(H, L, lo, hi):
    """lo <= x <= hi on the 64-bit column (H, L); bounds are Python ints
    within +-(10^18 + 1), or None for an open end."""
    if lo is not None and hi is not None and lo > hi:
        return ("lt", H, I32_MIN)
    parts = []
    lh = ll = hh = hl = None
    if lo is not None:
        lh, ll = _words(lo)
    if hi is not None:
        hh, hl = _words(hi)
    if lo is not None and hi is not None and lh == hh:
        return ("and", [("eq", H, lh), ("between", L, ll, hl)])
    parts.append(("between", H, lh if lo is not None else I32_MIN, hh if hi is not None else I32_MAX))
    if lo is not None:    # H > lh or L >= ll
        parts.append(("or", [("gt", H, lh), ("between", L, ll, I32_MAX)]))
    if hi is not None:    # H < hh or L <= hl
        parts.append(("or", [("lt", H, hh), ("between", L, I32_MIN, hl)]))
    return ("and", parts) if len(parts) > 1 else parts[0]


def _decimal64_leaf(scale, L, leaf):
    op, H = leaf[0], leaf[1]
    if op == "in":
        vals = sorted({v for v, e in (decimal_bound(x, scale, esc.EQ) for x in leaf[2]) if not e})
        if not vals:
            return ("lt", H, I32_MIN)
        groups = {}
        for v in vals:
            h, lo = _words(v)
            groups.setdefault(h, []).append(lo)
        # H in {h} and, for each h, (H != h or L in lows(h))
        parts = [("in", H, sorted(groups))]
        for h, lows in sorted(groups.items()):
            if len(groups) == 1:
                parts.append(("in", L, lows))
            else:
                parts.append(("or", [("lt", H, h), ("gt", H, h), ("in", L, lows)]))
        return ("and", parts)
    if op == "eq":
        v, empty = decimal_bound(leaf[2], scale, esc.EQ)
        return ("lt", H, I32_MIN) if empty else _range64(H, L, v, v)
    if op == "lt":
        return _range64(H, L, None, decimal_bound(leaf[2], scale, esc.LT)[0])
    if op == "gt":
        return _range64(H, L, decimal_bound(leaf[2], scale, esc.GT)[0], None)
    if op == "between":
        lo = decimal_bound(leaf[2], scale, esc.LT)[0] + 1
        hi = decimal_bound(leaf[3], scale, esc.GT)[0] - 1
        return _range64(H, L, lo, hi)
    raise ValueError(f"{op} is not a decimal comparison")


def lower(pred, types):
    """Rewrites leaves on typed columns; types maps a column to ("text",
    Dict), ("decimal", scale) (value * 10^scale in int32) or ("decimal64",
    scale, L) (value * 10^scale in int64 as the word columns H = this
    column and L, see split_words).  Other leaves are kept."""
    op = pred[0]
    if op in ("and", "or"):
        return (op, [lower(q, types) for q in pred[1]])
    if op == "udf" or pred[1] not in types:
        return pred
    kind, arg = types[pred[1]][0], types[pred[1]][1]
    if kind == "text":
        return _text_leaf(arg, pred)
    if kind == "decimal64":
        return _decimal64_leaf(arg, types[pred[1]][2], pred)
    return _decimal_leaf(arg, pred)
