"""TEXT and DECIMAL predicate columns, lowered onto their 4-byte storage.

Section 3 (Table 3) measures predicates on TEXT and DECIMAL(15,2) columns.
Here a TEXT column is stored as dictionary codes (rank in the dictionary's
byte-wise order) and a DECIMAL(p, s) column as value * 10^s in int32, or,
when its values exceed int32, in int64 held as two 32-bit word columns
(split_words, by the library's esc_decimal64_words).  The library rewrites
a predicate whose leaves compare typed columns with strings or decimal
literals into int32 leaves on the stored values (esc_lower_typed: code
ranges and sets, exact decimal bounds, 64-bit ranges on word columns),
which the ordinary compiler and kernels then evaluate; this module only
marshals the descriptions.

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


def _literal(v):
    """Text of a decimal literal given as a string or a decimal.Decimal
    (written out in positional notation)."""
    return format(v, "f") if isinstance(v, Decimal) else str(v)


def decimal_bound(literal, scale, op):
    """(bound, empty) of esc_decimal_bound for a literal given as a string
    or a decimal.Decimal."""
    b, e = ctypes.c_int64(), ctypes.c_int()
    esc.check(esc.lib().esc_decimal_bound(_literal(literal).encode(), int(scale), op, ctypes.byref(b),
                                          ctypes.byref(e)))
    return b.value, bool(e.value)


# ---------------------------------------------------------------- 64-bit decimals as two word columns
#
# A DECIMAL(15,2) value needs up to 10^15 stored units, beyond int32.  Such
# a column is stored as two 4-byte columns: H = the high 32 bits (signed)
# and L = the low 32 bits with the sign bit flipped (esc_decimal64_words), so
# that the order of the 64-bit values is the lexicographic order of (H, L);
# the library lowers every comparison on it to int32 leaves on H and L.

def split_words(x):
    """(H, L) int32 word columns of an int64 array (numpy, or a torch tensor
    on the host or the device, returned where it was)."""
    torch_in = not isinstance(x, np.ndarray)
    host = x.cpu().numpy() if torch_in else x
    v = np.ascontiguousarray(host, np.int64)
    hi = np.empty(v.shape, np.int32)
    lo = np.empty(v.shape, np.int32)
    esc.check(esc.lib().esc_decimal64_words(v.ctypes.data, v.size, hi.ctypes.data, lo.ctypes.data))
    if torch_in:
        import torch
        return torch.from_numpy(hi).to(x.device), torch.from_numpy(lo).to(x.device)
    return hi, lo


# ---------------------------------------------------------------- lowering (in the library)

_KIND = {"text": 1, "decimal": 2, "decimal64": 3}
_TYPED_OPS = {"eq": esc.EQ, "lt": esc.LT, "gt": esc.GT, "between": esc.BETWEEN, "in": esc.IN, "prefix": 8}
_NAMES = {esc.EQ: "eq", esc.LT: "lt", esc.GT: "gt", esc.BETWEEN: "between", esc.IN: "in"}


class ColType(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("scale", ctypes.c_int32), ("low_col", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("dict", ctypes.c_void_p)]


def _dtypes_of(schema):
    return list(schema.dtypes) if hasattr(schema, "dtypes") else list(schema)


def lower(pred, types, schema):
    """The predicate with its leaves on typed columns rewritten by the
    library (esc_lower_typed) into int32 leaves on their storage.  types maps
    a column to ("text", Dict), ("decimal", scale) (value * 10^scale in
    int32) or ("decimal64", scale, L) (value * 10^scale in int64 held as the
    word columns H = this column and L, see split_words); schema is an
    esc.Table or the column dtypes.  Other leaves are kept."""
    dtypes = _dtypes_of(schema)
    nodes, consts, lits, udfs = [], [], [], []

    def const(v, dt):
        c = esc.Const()
        c.dtype = dt
        if dt == esc.FLOAT32:
            c.v.bits = int(np.asarray(v, np.float32).view(np.uint32))
        else:
            c.v.i = int(v)
        consts.append(c)
        return len(consts) - 1

    def lit(v, kind):
        if kind == "text":
            lits.append(_c_str(v))
        else:
            lits.append(_literal(v).encode())
        return len(lits) - 1

    def walk(p):
        n = esc.Node()
        nodes.append(n)
        op = p[0]
        if op in ("and", "or"):
            n.op = esc.AND if op == "and" else esc.OR
            n.nchild = len(p[1])
            for q in p[1]:
                walk(q)
            return
        if op == "udf":   # kept as it is: the library copies the node, the description is put back
            n.op, n.cmp, n.k0 = esc.UDF, esc.EQ, const(0, esc.INT32)
            udfs.append(p)
            return
        c = p[1]
        n.col = c
        n.op = _TYPED_OPS[op]
        if c in types:
            kind = types[c][0]
            if op == "in":
                n.k0, n.k1 = len(lits), len(p[2])
                for v in p[2]:
                    lit(v, kind)
            elif op == "between":
                n.k0, n.k1 = lit(p[2], kind), lit(p[3], kind)
            else:
                n.k0 = lit(p[2], kind)
            return
        dt = dtypes[c]
        if op == "in":
            n.k0, n.k1 = len(consts), len(p[2])
            for v in p[2]:
                const(v, dt)
        elif op == "between":
            n.k0, n.k1 = const(p[2], dt), const(p[3], dt)
        else:
            n.k0 = const(p[2], dt)

    walk(pred)
    ct = (ColType * len(dtypes))()
    for c, t in types.items():
        ct[c].kind = _KIND[t[0]]
        if t[0] == "text":
            ct[c].dict = t[1].h.value
        else:
            ct[c].scale = int(t[1])
            if t[0] == "decimal64":
                ct[c].low_col = int(t[2])
    schema_t = esc.Table(0, dtypes, None)
    arr_n = (esc.Node * len(nodes))(*nodes)
    arr_c = (esc.Const * max(len(consts), 1))(*consts)
    arr_l = (ctypes.c_char_p * max(len(lits), 1))(*lits)
    cap_n, cap_c = 64 + 8 * len(nodes), 64 + 8 * len(consts) + 4 * len(lits)
    while True:
        out_n = (esc.Node * cap_n)()
        out_c = (esc.Const * cap_c)()
        nn, nc = ctypes.c_int(), ctypes.c_int()
        rc = esc.lib().esc_lower_typed(schema_t.h, ct, arr_n, len(nodes), arr_c, len(consts), arr_l, len(lits),
                                       out_n, cap_n, ctypes.byref(nn), out_c, cap_c, ctypes.byref(nc))
        if rc != esc.ERR_CAPACITY:
            esc.check(rc)
            break
        cap_n, cap_c = nn.value, nc.value
    return _unflatten(out_n[:nn.value], out_c[:nc.value], udfs)


def _unflatten(nodes, consts, udfs):
    """The description of a lowered node array (int32 and float32 constants)."""
    pos = 0
    it = iter(udfs)

    def val(k):
        c = consts[k]
        if c.dtype == esc.FLOAT32:
            return np.uint32(c.v.bits).view(np.float32)
        return int(c.v.i)

    def rec():
        nonlocal pos
        n = nodes[pos]
        pos += 1
        if n.op in (esc.AND, esc.OR):
            return ("and" if n.op == esc.AND else "or", [rec() for _ in range(n.nchild)])
        if n.op == esc.UDF:
            return next(it)
        name = _NAMES[n.op]
        if n.op == esc.IN:
            return (name, n.col, [val(n.k0 + i) for i in range(n.k1)])
        if n.op == esc.BETWEEN:
            return (name, n.col, val(n.k0), val(n.k1))
        return (name, n.col, val(n.k0))

    return rec()
