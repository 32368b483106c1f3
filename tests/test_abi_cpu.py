"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and the predicate compiler validates,
normalises and reports errors precisely."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "esc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(esc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = esc.lib()
    syms = declared_symbols()
    assert len(syms) >= 30
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing, missing
    assert L.esc_abi_version() == 8


@pytest.fixture(scope="module")
def schema():
    # int32, date32, float32, int32
    return esc.Table(1000, [dg.INT32, dg.DATE32, dg.FLOAT32, dg.INT32])


def rc_of(schema, spec):
    return esc.try_compile(schema, spec)


def test_valid_predicates_compile(schema):
    for spec in [("eq", 0, 5), ("between", 1, 8035, 9000), ("lt", 2, np.float32(1.5)),
                 ("in", 3, [1, 2, 3, 100]), ("and", [("eq", 0, 1), ("or", [("gt", 3, 4), ("eq", 1, 8100)])]),
                 ("udf", ("mod", ("add", ("mul", ("col", 0), ("const", 31)), ("col", 3)), ("const", 97)), ("gt", 5))]:
        assert rc_of(schema, spec) == esc.OK, esc.last_error()


@pytest.mark.parametrize("spec,want", [
    (("eq", 4, 5), esc.ERR_INVALID),                                # column out of range
    (("eq", -1, 5), esc.ERR_INVALID),
    (("in", 0, []), esc.ERR_INVALID),                               # empty IN
    (("udf", ("mod", ("col", 0), ("const", 0)), ("gt", 0)), esc.ERR_INVALID),   # mod 0
    (("udf", ("mod", ("col", 0), ("const", -3)), ("gt", 0)), esc.ERR_INVALID),  # negative modulus
    (("udf", ("shl", ("col", 0), ("const", 32)), ("gt", 0)), esc.ERR_INVALID),  # shift out of range
    (("udf", ("mod", ("col", 0), ("col", 3)), ("gt", 0)), esc.ERR_INVALID),     # non-constant modulus
    (("udf", ("add", ("col", 2), ("const", 1)), ("gt", 0)), esc.ERR_TYPE),      # float column in a udf
])
def test_compile_errors(schema, spec, want):
    assert rc_of(schema, spec) == want


def _compile_raw(schema, nodes, consts=(), udf=()):
    N = (esc.Node * max(len(nodes), 1))(*nodes)
    C = (esc.Const * max(len(consts), 1))(*consts)
    U = (esc.UdfInsn * max(len(udf), 1))(*udf)
    h = ctypes.c_void_p()
    rc = esc.lib().esc_compile_predicate(schema.h, N, len(nodes), C, len(consts), U, len(udf), ctypes.byref(h))
    if rc == 0:
        esc.lib().esc_pred_destroy(h)
    return rc


def _node(op, col=0, nchild=0, cmp=0, k0=0, k1=0, u0=0, u1=0):
    return esc.Node(op, col, nchild, cmp, k0, k1, u0, u1)


def _const(dt, v):
    c = esc.Const()
    c.dtype = dt
    if dt == esc.FLOAT32:
        c.v.f = v
    else:
        c.v.i = v
    return c


def test_raw_structure_errors(schema):
    k = [_const(esc.INT32, 3)]
    assert _compile_raw(schema, [_node(esc.EQ, 0)], k) == esc.OK
    assert _compile_raw(schema, [], k) == esc.ERR_INVALID                              # no nodes
    assert _compile_raw(schema, [_node(esc.AND, nchild=0)], k) == esc.ERR_INVALID      # childless AND
    assert _compile_raw(schema, [_node(esc.AND, nchild=2), _node(esc.EQ, 0)], k) == esc.ERR_INVALID  # truncated
    assert _compile_raw(schema, [_node(esc.EQ, 0), _node(esc.EQ, 0)], k) == esc.ERR_INVALID  # trailing node
    assert _compile_raw(schema, [_node(esc.EQ, 0, k0=5)], k) == esc.ERR_INVALID       # const index
    assert _compile_raw(schema, [_node(99, 0)], k) == esc.ERR_INVALID                  # bad op
    assert _compile_raw(schema, [_node(esc.EQ, 0, nchild=1)], k) == esc.ERR_INVALID    # leaf with children
    # dtype mismatches: float constant on an int column, int constant on a float column,
    # int32 constant on a date32 column
    assert _compile_raw(schema, [_node(esc.EQ, 0)], [_const(esc.FLOAT32, 1.0)]) == esc.ERR_TYPE
    assert _compile_raw(schema, [_node(esc.EQ, 2)], [_const(esc.INT32, 1)]) == esc.ERR_TYPE
    assert _compile_raw(schema, [_node(esc.EQ, 1)], [_const(esc.INT32, 1)]) == esc.ERR_TYPE
    # udf program must start with LOAD
    u = [esc.UdfInsn(esc.U_ADD, esc.U_CONST, 1)]
    assert _compile_raw(schema, [_node(esc.UDF, cmp=esc.GT, u0=0, u1=1)], k, u) == esc.ERR_INVALID
    u = [esc.UdfInsn(esc.U_LOAD, esc.U_COL, 0)]
    assert _compile_raw(schema, [_node(esc.UDF, cmp=esc.GT, u0=0, u1=1)], k, u) == esc.OK
    assert _compile_raw(schema, [_node(esc.UDF, cmp=esc.GT, u0=0, u1=2)], k, u) == esc.ERR_INVALID  # range
    assert _compile_raw(schema, [_node(esc.UDF, cmp=esc.AND, u0=0, u1=1)], k, u) == esc.ERR_INVALID  # cmp op


def test_null_arguments():
    L = esc.lib()
    h = ctypes.c_void_p()
    assert L.esc_compile_predicate(None, None, 0, None, 0, None, 0, ctypes.byref(h)) == esc.ERR_INVALID
    assert L.esc_count(None, None, None, None, 0, None, None) == esc.ERR_INVALID
    out = ctypes.c_uint64()
    assert L.esc_count(None, None, None, None, 0, None, ctypes.byref(out)) == esc.ERR_INVALID
    assert L.esc_pred_get_info(None, None) == esc.ERR_INVALID
    assert L.esc_count_begin(None, None, None, None, 0, None, 0) == esc.ERR_INVALID
    assert L.esc_count_begin(None, None, None, None, 0, None, -1) == esc.ERR_INVALID
    assert L.esc_count_end(None, 0, ctypes.byref(out)) == esc.ERR_INVALID


def test_table_create_errors():
    L = esc.lib()
    h = ctypes.c_void_p()
    dt = np.array([0, 2], np.int32)
    ptrs = (ctypes.c_void_p * 2)(0x10000, 0x10008)      # second column misaligned
    assert L.esc_table_create(10, 2, dt.ctypes.data, ptrs, ctypes.byref(h)) == esc.ERR_ALIGN
    assert L.esc_table_create(-1, 2, dt.ctypes.data, None, ctypes.byref(h)) == esc.ERR_INVALID
    assert L.esc_table_create(2**31, 2, dt.ctypes.data, None, ctypes.byref(h)) == esc.ERR_INVALID
    assert L.esc_table_create(10, 0, dt.ctypes.data, None, ctypes.byref(h)) == esc.ERR_INVALID
    bad = np.array([0, 7], np.int32)
    assert L.esc_table_create(10, 2, bad.ctypes.data, None, ctypes.byref(h)) == esc.ERR_INVALID


def test_scan_on_schema_only_table_is_rejected(schema):
    p = esc.Pred(schema, ("eq", 0, 1))
    out = ctypes.c_uint64()
    # a fake (never dereferenced) context pointer is enough to reach the table check
    rc = esc.lib().esc_count(ctypes.c_void_p(16), schema.h, p.h, ctypes.c_void_p(256), 4096, None, ctypes.byref(out))
    assert rc == esc.ERR_INVALID
    assert "schema-only" in esc.last_error()
    rc = esc.lib().esc_count_begin(ctypes.c_void_p(16), schema.h, p.h, ctypes.c_void_p(256), 4096, None, 3)
    assert rc == esc.ERR_INVALID and "schema-only" in esc.last_error()
    rc = esc.lib().esc_count_begin(ctypes.c_void_p(16), schema.h, p.h, ctypes.c_void_p(256), 4096, None, 64)
    assert rc == esc.ERR_INVALID and "slot" in esc.last_error()


def test_normalisation_info(schema):
    info = lambda s: esc.Pred(schema, s).info()
    # OR over AND distributes: (a AND b) OR c -> (a OR c) AND (b OR c)
    i = info(("or", [("and", [("eq", 0, 1), ("eq", 3, 2)]), ("gt", 1, 9000)]))
    assert i["nclauses"] == 2 and i["ncols"] == 3 and i["constant"] == 0
    assert i["col_mask"] == 0b1011
    # constant folding
    assert info(("lt", 0, -2**31))["constant"] == -1
    assert info(("gt", 0, 2**31 - 1))["constant"] == -1
    assert info(("between", 0, -2**31, 2**31 - 1))["constant"] == 1
    assert info(("between", 0, 5, 4))["constant"] == -1
    assert info(("lt", 2, np.float32(np.nan)))["constant"] == -1
    assert info(("lt", 2, np.float32(-np.inf)))["constant"] == -1
    assert info(("gt", 2, np.float32(np.inf)))["constant"] == -1
    assert info(("in", 2, [np.float32(np.nan)]))["constant"] == -1
    assert info(("and", [("eq", 0, 1), ("lt", 0, -2**31)]))["constant"] == -1
    assert info(("or", [("eq", 0, 1), ("between", 3, -2**31, 2**31 - 1)]))["constant"] == 1
    # float ranges never fold to true (NaN rows fail them)
    assert info(("between", 2, np.float32(-np.inf), np.float32(np.inf)))["constant"] == 0
    # the Section 1 example: 4 clauses over B, C, D
    p = dg.pred_plain(dg.table_plain(100, seed=1), 3)
    i = esc.Pred(esc.Table(100, [dg.INT32] * 4), p).info()
    assert i["nclauses"] == 4 and i["ncols"] == 3 and i["col_mask"] == 0b1110


def test_limits(schema):
    wide = esc.Table(10, [dg.INT32] * 12)
    nine = ("and", [("eq", c, 1) for c in range(9)])
    assert esc.try_compile(wide, nine) == esc.ERR_UNSUPPORTED        # more than 8 columns
    eight = ("and", [("eq", c, 1) for c in range(8)])
    assert esc.try_compile(wide, eight) == esc.OK
    big_in = ("in", 0, list(range(0, 65 * 1000, 1000)))              # 65 distinct sparse constants
    assert esc.try_compile(schema, big_in) == esc.ERR_UNSUPPORTED
    # OR of 6 two-leaf ANDs distributes into 64 clauses
    blow = ("or", [("and", [("eq", 0, i), ("eq", 3, i)]) for i in range(6)])
    assert esc.try_compile(schema, blow) == esc.ERR_UNSUPPORTED


def test_ctx_without_gpu():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    h = ctypes.c_void_p()
    assert esc.lib().esc_ctx_create(0, ctypes.byref(h)) == esc.ERR_HIP


def test_in_slot_tables(schema, monkeypatch):
    """IN-lists of three or more sparse keys become slot-table lookups when a
    6-bit field, a bitmap or a multiplicative hash separates the keys;
    otherwise, or when the constant pool cannot hold another 64-entry table,
    they stay compare lists."""
    info = lambda s: esc.Pred(schema, s).info()
    assert info(("in", 0, [5, 1000, 77777]))["nhashed"] == 1
    assert info(("in", 0, [5, 1000]))["nhashed"] == 0              # two compares are cheaper
    assert info(("in", 0, list(range(0, 640, 10))))["nhashed"] == 1  # 64 keys, one per slot
    # 0, 1 and 65536: every cyclic 6-bit field misses bit 0 or bit 16, so one
    # pair of keys always shares a field value, and they span more than a
    # bitmap; a multiplicative hash would separate them, but three compares
    # cost less than a multiply per row
    assert info(("in", 0, [0, 1, 65536]))["nhashed"] == 0
    # sixteen keys made of bits 0, 8, 16 and 24: a 6-bit field sees at most
    # one of those bits (two field values for sixteen keys); the top bits of
    # a product with an odd multiplier separate them (from eight keys on)
    spread = [(i & 1) | (i >> 1 & 1) << 8 | (i >> 2 & 1) << 16 | (i >> 3 & 1) << 24 for i in range(16)]
    assert info(("in", 0, spread))["nhashed"] == 1
    assert info(("in", 0, spread[:8]))["nhashed"] == 1
    assert info(("in", 0, spread[:7]))["nhashed"] == 0
    # no field separates 0, 2, 66, 130 (they need bits 1, 6 and 7), but they
    # span less than 2048: a bitmap; one more key 2048 away: a compare list
    assert info(("in", 0, [0, 2, 66, 130]))["nhashed"] == 1
    assert info(("in", 0, [0, 2, 66, 130, 2047]))["nhashed"] == 1
    assert info(("in", 0, [0, 2, 66, 130, 2048]))["nhashed"] == 0
    # 64 keys spread over the int range: no hash of either family is a
    # perfect one, and they span more than a bitmap
    wide = [int(v) for v in np.random.default_rng(9).choice(2**31 - 1, 64, replace=False)]
    assert info(("in", 0, wide))["nhashed"] == 0
    # float lists: a zero constant needs both zero patterns (two slots)
    assert info(("in", 2, [np.float32(v) for v in (0.0, 2.5, -7.0)]))["nhashed"] == 1
    # pool budget (256 constants): 64 + 4 * 3 as lists leave 180, and each
    # table takes 61 more, so two of the four short lists become tables
    # (compiled as written: intersecting the two lists on column 0 would
    # prove the conjunction empty)
    monkeypatch.setenv("ESC_SIMPLIFY", "0")
    lists = [("in", c, [10 + i, 5000 + i, 900000 + i]) for i, c in enumerate((0, 1, 3, 0))]
    big = ("in", 1, [7 * i * i + 3 for i in range(64)])
    pred = ("and", lists + [big])
    i = info(pred)
    assert i["nhashed"] == (1 if info(big)["nhashed"] else 0) + 2
    monkeypatch.setenv("ESC_IN_HASH_MIN", "0")
    assert info(pred)["nhashed"] == 0
    assert info(("in", 0, [5, 1000, 77777]))["nhashed"] == 0


def test_autotune_cache_file_skips_bad_entries(tmp_path):
    """Tuning-cache lines whose options a batch would not accept (rows per
    thread other than 8 or 16, a block other than 256, negative group, chunk
    or blocks per CU, max_cols other than 0, 4, 6 or 8, missing or extra
    fields) are skipped, not installed."""
    L = esc.lib()
    f = tmp_path / "tune.txt"
    f.write_text("k1 256 16 0 0 0\n"
                 "k2 256 0 16 131072 2\n"       # rows per thread 0 (a division by zero when planning)
                 "k3 256 8 -1 0 0\n"
                 "k4 512 8 0 0 0\n"
                 "k5 256 8 0 -5 0\n"
                 "k6 256 16 8 1048576 -1\n"
                 "junk\n"
                 "\n"
                 "k7 256 8 16 131072 2\n"
                 "k8 256 8 0 0 0 9\n"          # max_cols 9
                 "k9 256 16 0 0 0 4\n"
                 "k10 256 16 0 0 2 6\n"
                 "k11 256 16 0 0 2 5\n"        # max_cols 5
                 "k12 256 16 0 0 2 8 1\n")     # an extra field
    acc, rej = ctypes.c_int(-1), ctypes.c_int(-1)
    assert L.esc_batch_tune_cache_load(str(f).encode(), ctypes.byref(acc), ctypes.byref(rej)) == esc.OK
    assert (acc.value, rej.value) == (4, 9)
    assert L.esc_batch_tune_cache_load(str(tmp_path / "missing").encode(), None, None) == esc.ERR_INVALID


@pytest.mark.parametrize("spec,insns,const", [
    (("and", [("lt", 0, 50), ("gt", 0, 10)]), 1, 0),                         # one range
    (("and", [("lt", 0, 5), ("gt", 0, 10)]), 0, -1),                         # contradiction
    (("and", [("in", 3, [1, 5, 9, 40]), ("lt", 3, 30)]), 1, 0),              # IN filtered by the range
    (("and", [("in", 0, [1, 2, 3]), ("in", 0, [4, 5])]), 0, -1),             # disjoint IN-lists
    (("and", [("gt", 0, 100), ("or", [("lt", 0, 50), ("eq", 3, 3)])]), 2, 0),  # OR leaf that cannot hold
    (("and", [("between", 0, 10, 20), ("or", [("lt", 0, 50), ("eq", 3, 3)])]), 1, 0),  # OR that always holds
    (("and", [("lt", 2, np.float32(0.0)), ("gt", 2, np.float32(-0.0))]), 0, -1),  # no float is < 0 and > -0
    (("and", [("between", 2, np.float32(-0.0), np.float32(0.0)), ("eq", 2, np.float32(0.0))]), 1, 0),
    (("and", [("eq", 1, 9000), ("between", 1, 8000, 9500), ("eq", 0, 3)]), 2, 0),
    (("and", [("gt", 0, 5), ("or", [("lt", 0, 3), ("lt", 0, 1)])]), 0, -1),  # every OR leaf excluded
])
def test_conjunct_simplification(schema, spec, insns, const, monkeypatch):
    """Conjuncts on one column are intersected at compile time (exact: the
    GPU parity tests compare the simplified programs' counts with the
    oracle, which evaluates the predicate as written)."""
    info = esc.Pred(schema, spec).info()
    assert (info["ninsns"], info["constant"]) == (insns, const), info
    monkeypatch.setenv("ESC_SIMPLIFY", "0")
    off = esc.Pred(schema, spec).info()
    assert off["ninsns"] >= insns and (off["constant"] == 0 or const == off["constant"])
