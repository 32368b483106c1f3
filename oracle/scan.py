"""Python side of the CPU scan oracle (esc_oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline of the benchmark, never by the product path.

`to_sexpr` writes a predicate description (the nested-tuple format of the
input generators) in the oracle's own S-expression syntax; the C oracle
parses that text itself, so a flattening bug in the product binding cannot
be shared with the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "esc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FLOAT32 = 2


def build(force=False):
    """Compile the oracle with the host C compiler (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-Wall", "-Wextra", "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        vp = ctypes.c_void_p
        L.oracle_count.argtypes = [ctypes.c_int64, ctypes.c_int, vp, vp, ctypes.c_char_p, vp]
        L.oracle_materialize.argtypes = [ctypes.c_int64, ctypes.c_int, vp, vp, ctypes.c_char_p,
                                         ctypes.c_int, vp, vp, vp, ctypes.c_uint64, vp]
        L.oracle_eval_rows.argtypes = [ctypes.c_int64, ctypes.c_int, vp, vp, ctypes.c_char_p, vp]
        L.oracle_check.argtypes = [ctypes.c_int, vp, ctypes.c_char_p]
        L.oracle_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


# ------------------------------------------------------------ predicate text

def _k(v, is_float):
    if is_float:
        return "fx%08x" % int(np.array(v, dtype=np.float32).view(np.uint32))
    v = int(v)
    if not -2**31 <= v < 2**31:
        raise ValueError("int32 constant out of range: %r" % v)
    return str(v)


def _expr(e):
    if e[0] == "col":
        return "(col %d)" % e[1]
    if e[0] == "const":
        return "(const %s)" % _k(e[1], False)
    return "(%s %s %s)" % (e[0], _expr(e[1]), _expr(e[2]))


def _test(t):
    if t[0] == "in":
        return "(in %s)" % " ".join(_k(v, False) for v in t[1])
    return "(%s %s)" % (t[0], " ".join(_k(v, False) for v in t[1:]))


def to_sexpr(p, dtypes):
    op = p[0]
    if op in ("and", "or"):
        return "(%s %s)" % (op, " ".join(to_sexpr(q, dtypes) for q in p[1]))
    if op == "udf":
        return "(udf %s %s)" % (_expr(p[1]), _test(p[2]))
    c = p[1]
    fl = dtypes[c] == FLOAT32
    if op == "in":
        return "(in %d %s)" % (c, " ".join(_k(v, fl) for v in p[2]))
    return "(%s %d %s)" % (op, c, " ".join(_k(v, fl) for v in p[2:]))


# ------------------------------------------------------------ calls

def _cols(table):
    cols = [np.ascontiguousarray(c if isinstance(c, np.ndarray) else c.cpu().numpy()) for c in table.cols]
    for c in cols:
        if c.dtype.itemsize != 4 or len(c) != table.nrows:
            raise ValueError("columns must be 4-byte arrays of nrows elements")
    ptrs = (ctypes.c_void_p * len(cols))(*[c.ctypes.data for c in cols])
    dts = np.asarray(table.dtypes, dtype=np.int32)
    return cols, ptrs, dts


def _fail():
    raise OracleError(lib().oracle_error().decode())


def count(table, pred) -> int:
    """Exact COUNT(*) of the rows of `table` satisfying `pred`."""
    cols, ptrs, dts = _cols(table)
    out = np.zeros(1, np.uint64)
    text = to_sexpr(pred, table.dtypes).encode()
    if lib().oracle_count(table.nrows, len(cols), dts.ctypes.data, ptrs, text, out.ctypes.data) != 0:
        _fail()
    return int(out[0])


def eval_rows(table, pred) -> np.ndarray:
    """Truth value of `pred` on every row, as a bool array."""
    cols, ptrs, dts = _cols(table)
    mask = np.zeros(max(table.nrows, 1), np.uint8)
    text = to_sexpr(pred, table.dtypes).encode()
    if lib().oracle_eval_rows(table.nrows, len(cols), dts.ctypes.data, ptrs, text, mask.ctypes.data) != 0:
        _fail()
    return mask[: table.nrows].astype(bool)


def materialize(table, pred, proj, capacity=None):
    """(count, rowids, [projected columns]) of the selection, in row order.
    At most `capacity` rows are returned (default: all)."""
    cols, ptrs, dts = _cols(table)
    text = to_sexpr(pred, table.dtypes).encode()
    if capacity is None:
        capacity = count(table, pred)
    rowids = np.zeros(max(capacity, 1), np.int32)
    outs = [np.zeros(max(capacity, 1), cols[j].dtype) for j in proj]
    optrs = (ctypes.c_void_p * max(len(outs), 1))(*[o.ctypes.data for o in outs])
    pj = np.asarray(proj, dtype=np.int32)
    cnt = np.zeros(1, np.uint64)
    rc = lib().oracle_materialize(table.nrows, len(cols), dts.ctypes.data, ptrs, text, len(proj),
                                  pj.ctypes.data, rowids.ctypes.data, optrs, capacity, cnt.ctypes.data)
    if rc < 0:
        _fail()
    c = int(cnt[0])
    k = min(c, capacity)
    return c, rowids[:k], [o[:k] for o in outs]


def check(dtypes, text) -> bool:
    dts = np.asarray(dtypes, dtype=np.int32)
    return lib().oracle_check(len(dtypes), dts.ctypes.data, text.encode()) == 0


def count_many(table, preds):
    return [count(table, p) for p in preds]
