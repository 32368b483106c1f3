"""Thin ctypes binding of libesc.so (include/esc.h).

Argument marshalling only: predicate descriptions are flattened into the
esc_node / esc_const / esc_udf_insn arrays of the C ABI, torch tensors are
passed as raw device pointers and streams as hipStream_t handles.  Every step
of the scan, the batched count and the MLP runs in the library's kernels; if
the library is not built this module raises on import of the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libesc.so")

INT32, DATE32, FLOAT32 = 0, 1, 2
OK, ERR_INVALID, ERR_TYPE, ERR_CAPACITY, ERR_ALIGN, ERR_HIP, ERR_OOM, ERR_UNSUPPORTED, ERR_TIMEOUT = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "TYPE", -3: "CAPACITY", -4: "ALIGN", -5: "HIP", -6: "OOM",
                -7: "UNSUPPORTED", -8: "TIMEOUT"}

AND, OR, EQ, LT, GT, BETWEEN, IN, UDF = range(8)
DICT_PREFIX = 100
_OPS = {"and": AND, "or": OR, "eq": EQ, "lt": LT, "gt": GT, "between": BETWEEN, "in": IN, "udf": UDF}
U_LOAD, U_ADD, U_SUB, U_MUL, U_MOD, U_AND, U_OR, U_XOR, U_SHL, U_SHR = range(10)
_UOPS = {"add": U_ADD, "sub": U_SUB, "mul": U_MUL, "mod": U_MOD, "band": U_AND, "bor": U_OR,
         "bxor": U_XOR, "shl": U_SHL, "shr": U_SHR}
U_COL, U_CONST = 0, 1
MLP_NPARAMS = 148481
MAX_PROJ = 8
MAX_CONJ = 32


class EscError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"esc status {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("col", ctypes.c_int32), ("nchild", ctypes.c_int32),
                ("cmp", ctypes.c_int32), ("k0", ctypes.c_int32), ("k1", ctypes.c_int32),
                ("u0", ctypes.c_int32), ("u1", ctypes.c_int32)]


class Value(ctypes.Union):
    _fields_ = [("i", ctypes.c_int32), ("f", ctypes.c_float), ("bits", ctypes.c_uint32)]


class Const(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("v", Value)]


class UdfInsn(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("src", ctypes.c_int32), ("arg", ctypes.c_int32)]


class PredInfo(ctypes.Structure):
    _fields_ = [("nclauses", ctypes.c_int32), ("ninsns", ctypes.c_int32), ("ncols", ctypes.c_int32),
                ("constant", ctypes.c_int32), ("col_mask", ctypes.c_uint64), ("nhashed", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class CostModel(ctypes.Structure):
    _fields_ = [("scan_bytes_per_s", ctypes.c_double), ("fixed_s", ctypes.c_double),
                ("sparse_row_s", ctypes.c_double), ("dense_fraction", ctypes.c_double),
                ("dense_bytes_per_s", ctypes.c_double), ("dense_row_s", ctypes.c_double),
                ("tmp_bytes_per_s", ctypes.c_double)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("autotune", ctypes.c_int32), ("block", ctypes.c_int32), ("rows_per_thread", ctypes.c_int32),
                ("group", ctypes.c_int32), ("chunk_rows", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("max_preds", ctypes.c_int32), ("max_cols", ctypes.c_int32)]


WS_COUNT, WS_MATERIALIZE, WS_CONJUNCTS = 0, 1, 2   # esc_workspace_size kinds
ABI_VERSION = 8   # esc.h's ESC_ABI_VERSION for the struct layouts below

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1901_01488_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        P = ctypes.POINTER
        sig = {
            "esc_last_error": ([], ctypes.c_char_p),
            "esc_abi_version": ([], ctypes.c_int),
            "esc_ctx_create": ([ctypes.c_int, P(vp)], ctypes.c_int),
            "esc_ctx_destroy": ([vp], ctypes.c_int),
            "esc_ctx_num_cus": ([vp, P(ctypes.c_int)], ctypes.c_int),
            "esc_table_create": ([i64, ctypes.c_int, vp, vp, P(vp)], ctypes.c_int),
            "esc_table_destroy": ([vp], ctypes.c_int),
            "esc_compile_predicate": ([vp, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, P(vp)], ctypes.c_int),
            "esc_pred_destroy": ([vp], ctypes.c_int),
            "esc_pred_get_info": ([vp, P(PredInfo)], ctypes.c_int),
            "esc_workspace_size": ([vp, ctypes.c_int, P(ctypes.c_size_t)], ctypes.c_int),
            "esc_workspace_init": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "esc_count": ([vp, vp, vp, vp, ctypes.c_size_t, vp, P(u64)], ctypes.c_int),
            "esc_count_async": ([vp, vp, vp, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
            "esc_count_begin": ([vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_int], ctypes.c_int),
            "esc_count_end": ([vp, ctypes.c_int, P(u64)], ctypes.c_int),
            "esc_materialize": ([vp, vp, vp, vp, ctypes.c_int, vp, vp, u64, vp, ctypes.c_size_t, vp, P(u64)],
                                ctypes.c_int),
            "esc_materialize_async": ([vp, vp, vp, vp, ctypes.c_int, vp, vp, u64, vp, ctypes.c_size_t, vp, vp],
                                      ctypes.c_int),
            "esc_materialize_noalloc": ([vp, vp, vp, vp, ctypes.c_int, vp, vp, u64, vp, vp], ctypes.c_int),
            "esc_count_conjuncts": ([vp, vp, vp, vp, ctypes.c_size_t, vp, ctypes.c_int, vp, vp, P(ctypes.c_int)],
                                    ctypes.c_int),
            "esc_batch_workspace_size": ([vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, P(BatchOpts),
                                          P(ctypes.c_size_t)], ctypes.c_int),
            "esc_batch_create": ([vp, vp, ctypes.c_int, vp, vp, ctypes.c_int, P(BatchOpts), vp, ctypes.c_size_t, vp,
                                  P(vp)], ctypes.c_int),
            "esc_batch_tune_cache_load": ([ctypes.c_char_p, P(ctypes.c_int), P(ctypes.c_int)], ctypes.c_int),
            "esc_lower_typed": ([vp, vp, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int, vp, ctypes.c_int,
                                 P(ctypes.c_int), vp, ctypes.c_int, P(ctypes.c_int)], ctypes.c_int),
            "esc_decimal64_words": ([vp, i64, vp, vp], ctypes.c_int),
            "esc_batch_update": ([vp, vp, vp, ctypes.c_int, vp], ctypes.c_int),
            "esc_batch_count": ([vp, vp, vp], ctypes.c_int),
            "esc_batch_get_opts": ([vp, P(BatchOpts)], ctypes.c_int),
            "esc_batch_destroy": ([vp], ctypes.c_int),
            "esc_featurize": ([vp, vp, vp, vp, ctypes.c_int, vp, ctypes.c_int, vp], ctypes.c_int),
            "esc_catalog_create": ([vp, vp, vp, vp, ctypes.c_int, P(vp)], ctypes.c_int),
            "esc_catalog_destroy": ([vp], ctypes.c_int),
            "esc_featurize_catalog": ([vp, vp, ctypes.c_int, vp], ctypes.c_int),
            "esc_mlp_state_bytes": ([], ctypes.c_size_t),
            "esc_mlp_workspace_bytes": ([ctypes.c_int], ctypes.c_size_t),
            "esc_mlp_create": ([vp, vp, ctypes.c_size_t, P(vp)], ctypes.c_int),
            "esc_mlp_destroy": ([vp], ctypes.c_int),
            "esc_mlp_set_params": ([vp, vp], ctypes.c_int),
            "esc_mlp_get_params": ([vp, vp], ctypes.c_int),
            "esc_mlp_get_state": ([vp, vp, vp, vp, P(i64)], ctypes.c_int),
            "esc_mlp_set_state": ([vp, vp, vp, vp, i64], ctypes.c_int),
            "esc_mlp_save": ([vp, ctypes.c_char_p], ctypes.c_int),
            "esc_mlp_load": ([vp, ctypes.c_char_p], ctypes.c_int),
            "esc_mlp_predict": ([vp, vp, i64, vp, vp], ctypes.c_int),
            "esc_mlp_gradients": ([vp, vp, vp, i64, vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "esc_mlp_train": ([vp, vp, vp, vp, i64, ctypes.c_int, ctypes.c_float, vp, ctypes.c_size_t, vp, vp],
                              ctypes.c_int),
            "esc_gate_pushdown": ([vp, vp, ctypes.c_int, ctypes.c_double, ctypes.c_double, i64, vp], ctypes.c_int),
            "esc_gate_join_pair": ([ctypes.c_float, i64, ctypes.c_float, i64, ctypes.c_double, vp], ctypes.c_int),
            "esc_gate_join_pairs": ([vp, i64, vp, i64, ctypes.c_int, ctypes.c_double, ctypes.c_double, vp],
                                    ctypes.c_int),
            "esc_ctx_dense_fraction": ([vp, vp], ctypes.c_int),
            "esc_dict_create": ([vp, ctypes.c_int, vp], ctypes.c_int),
            "esc_dict_destroy": ([vp], ctypes.c_int),
            "esc_dict_size": ([vp, vp], ctypes.c_int),
            "esc_dict_code": ([vp, ctypes.c_char_p, vp], ctypes.c_int),
            "esc_dict_string": ([vp, ctypes.c_int32, vp], ctypes.c_int),
            "esc_dict_range": ([vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_char_p, vp, vp], ctypes.c_int),
            "esc_decimal_bound": ([ctypes.c_char_p, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
            "esc_hash_table_bytes": ([i64, vp], ctypes.c_int),
            "esc_hash_build": ([vp, vp, i64, vp, ctypes.c_size_t, vp], ctypes.c_int),
            "esc_join_count": ([vp, vp, vp, vp, vp, ctypes.c_int, vp, ctypes.c_size_t, vp, vp], ctypes.c_int),
            "esc_policy_keep": ([vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp],
                                ctypes.c_int),
            "esc_policy_thresholds": ([vp, i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        if L.esc_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.esc_abi_version()}, this binding needs "
                              f"{ABI_VERSION}: rebuild it with `python -m paper_1901_01488_amd.build`")
        _lib = L
    return _lib


def check(rc):
    if rc != OK:
        raise EscError(rc, lib().esc_last_error().decode())
    return rc


def last_error():
    return lib().esc_last_error().decode()


# ------------------------------------------------------------------ predicates

def flatten(pred, dtypes):
    """Pre-order esc_node array, typed constants and udf program of a
    predicate description (see datagen's module docstring)."""
    nodes, consts, udf = [], [], []

    def const(v, dt):
        c = Const()
        c.dtype = dt
        if dt == FLOAT32:
            c.v.bits = int(np.asarray(v, np.float32).view(np.uint32))
        else:
            c.v.i = int(v)
        consts.append(c)
        return len(consts) - 1

    def cmp_consts(op, args, dt):
        if op == "in":
            k0 = len(consts)
            for v in args[0]:
                const(v, dt)
            return k0, len(args[0])
        if op == "between":
            return const(args[0], dt), const(args[1], dt)
        return const(args[0], dt), 0

    def udf_prog(e):
        # left-deep chain: (op, E, leaf) ... (col c) | (const k)
        chain = []
        while e[0] not in ("col", "const"):
            chain.append(e)
            e = e[1]
        prog = [(U_LOAD, U_COL if e[0] == "col" else U_CONST, int(e[1]))]
        for op in reversed(chain):
            rhs = op[2]
            if rhs[0] not in ("col", "const"):
                raise ValueError("udf operands must be columns or constants (left-deep expressions)")
            prog.append((_UOPS[op[0]], U_COL if rhs[0] == "col" else U_CONST, int(rhs[1])))
        return prog

    def walk(p):
        op = p[0]
        n = Node()
        n.op = _OPS[op]
        nodes.append(n)
        if op in ("and", "or"):
            n.nchild = len(p[1])
            for q in p[1]:
                walk(q)
            return
        if op == "udf":
            prog = udf_prog(p[1])
            n.u0, n.u1 = len(udf), len(prog)
            for (o, s, a) in prog:
                udf.append(UdfInsn(o, s, a))
            t = p[2]
            n.cmp = _OPS[t[0]]
            n.k0, n.k1 = cmp_consts(t[0], t[1:], INT32)
            return
        n.col = p[1]
        dt = dtypes[p[1]] if 0 <= p[1] < len(dtypes) else INT32   # the library rejects the column
        n.k0, n.k1 = cmp_consts(op, p[2:], dt)

    walk(pred)
    return ((Node * len(nodes))(*nodes), len(nodes), (Const * max(len(consts), 1))(*consts), len(consts),
            (UdfInsn * max(len(udf), 1))(*udf), len(udf))


class Table:
    """A table descriptor; device columns (torch tensors of 4-byte dtype) or
    schema only (cols=None)."""

    def __init__(self, nrows, dtypes, cols=None):
        self.nrows = int(nrows)
        self.dtypes = list(dtypes)
        self.cols = cols
        dt = np.asarray(self.dtypes, np.int32)
        self._dt = dt
        ptrs = None
        if cols is not None:
            ptrs = (ctypes.c_void_p * len(cols))(*[c.data_ptr() for c in cols])
        self._ptrs = ptrs
        h = ctypes.c_void_p()
        check(lib().esc_table_create(self.nrows, len(self.dtypes), dt.ctypes.data, ptrs, ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_table_destroy(self.h)
            self.h = None


class Pred:
    def __init__(self, schema: Table, spec):
        nodes, nn, consts, nc, udf, nu = flatten(spec, schema.dtypes)
        h = ctypes.c_void_p()
        check(lib().esc_compile_predicate(schema.h, nodes, nn, consts, nc, udf, nu, ctypes.byref(h)))
        self.h = h
        self.spec = spec

    def info(self):
        i = PredInfo()
        check(lib().esc_pred_get_info(self.h, ctypes.byref(i)))
        return {"nclauses": i.nclauses, "ninsns": i.ninsns, "ncols": i.ncols, "constant": i.constant,
                "col_mask": i.col_mask, "nhashed": i.nhashed}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_pred_destroy(self.h)
            self.h = None


def compile_predicate(schema: Table, spec) -> Pred:
    return Pred(schema, spec)


def try_compile(schema: Table, spec):
    """Status code of compiling spec (no exception)."""
    nodes, nn, consts, nc, udf, nu = flatten(spec, schema.dtypes)
    h = ctypes.c_void_p()
    rc = lib().esc_compile_predicate(schema.h, nodes, nn, consts, nc, udf, nu, ctypes.byref(h))
    if rc == OK:
        lib().esc_pred_destroy(h)
    return rc


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    def __init__(self, device=0):
        h = ctypes.c_void_p()
        check(lib().esc_ctx_create(device, ctypes.byref(h)))
        self.h = h
        self.device = device
        self._ws = {}

    def num_cus(self):
        n = ctypes.c_int()
        check(lib().esc_ctx_num_cus(self.h, ctypes.byref(n)))
        return n.value

    def hash_table(self, keys, stream=None):
        """Device hash table (a uint8 tensor) of an int32 device key tensor."""
        import torch
        nb = ctypes.c_size_t()
        check(lib().esc_hash_table_bytes(int(keys.numel()), ctypes.byref(nb)))
        tab = torch.empty(nb.value, dtype=torch.uint8, device=keys.device)
        check(lib().esc_hash_build(self.h, ctypes.c_void_p(keys.data_ptr()) if keys.numel() else None,
                                   int(keys.numel()), ctypes.c_void_p(tab.data_ptr()), nb.value,
                                   _stream_handle(stream)))
        return tab

    def join_count(self, probe: Table, key_cols, tables, stream=None) -> int:
        """Rows of the star join of `probe` (key_cols[j] against tables[j])."""
        kc = np.asarray(key_cols, np.int32)
        ptrs = (ctypes.c_void_p * len(tables))(*[t.data_ptr() for t in tables])
        sizes = (ctypes.c_size_t * len(tables))(*[t.numel() for t in tables])
        out = ctypes.c_uint64()
        ws = self.workspace(probe, WS_COUNT, key="count")
        check(lib().esc_join_count(self.h, probe.h, kc.ctypes.data, ptrs, sizes, len(tables),
                                   ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream),
                                   ctypes.byref(out)))
        return out.value

    def dense_fraction(self):
        """Tile density from which the materialization reads projected columns whole."""
        v = ctypes.c_double()
        check(lib().esc_ctx_dense_fraction(self.h, ctypes.byref(v)))
        return v.value

    def workspace(self, table: Table, kind=WS_MATERIALIZE, key=None):
        """A zero-filled device workspace of the given kind (WS_COUNT,
        WS_MATERIALIZE or WS_CONJUNCTS; a bool means materialize or not) big
        enough for `table` (cached per key)."""
        import torch
        nb = ctypes.c_size_t()
        check(lib().esc_workspace_size(table.h, int(kind), ctypes.byref(nb)))
        # counts and materializations share one default workspace (a count
        # on a materialization-sized workspace leaves its tiles for the next
        # materialization of the same predicate)
        k = key if key is not None else ("default" if int(kind) in (WS_COUNT, WS_MATERIALIZE) else ("default", int(kind)))
        ws = self._ws.get(k)
        if ws is None or ws.numel() < nb.value:
            ws = torch.zeros(nb.value, dtype=torch.uint8, device=f"cuda:{self.device}")
            # a new allocation may sit at the address of a freed workspace:
            # drop whatever the library remembers about that address
            check(lib().esc_workspace_init(self.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(), None))
            self._ws[k] = ws
        return ws

    def count(self, table: Table, pred: Pred, ws=None, stream=None) -> int:
        ws = self.workspace(table, False) if ws is None else ws
        out = ctypes.c_uint64()
        check(lib().esc_count(self.h, table.h, pred.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                              _stream_handle(stream), ctypes.byref(out)))
        return out.value

    def count_async(self, table: Table, pred: Pred, dev_out, ws, stream=None):
        check(lib().esc_count_async(self.h, table.h, pred.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_handle(stream), ctypes.c_void_p(dev_out.data_ptr())))

    def count_begin(self, table: Table, pred: Pred, ws, slot, stream=None):
        """Enqueues the count; its result waits in the context's host slot."""
        check(lib().esc_count_begin(self.h, table.h, pred.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                    _stream_handle(stream), int(slot)))

    def count_end(self, slot) -> int:
        """Waits for the count begun on this slot and returns it."""
        out = ctypes.c_uint64()
        check(lib().esc_count_end(self.h, int(slot), ctypes.byref(out)))
        return out.value

    def materialize(self, table: Table, pred: Pred, proj, rowids, outs, capacity, ws=None, stream=None,
                    allow_overflow=False):
        """Returns the count; rowids/outs are caller-owned device tensors."""
        ws = self.workspace(table, True) if ws is None else ws
        pj = np.asarray(proj, np.int32)
        optrs = (ctypes.c_void_p * max(len(outs), 1))(*[o.data_ptr() for o in outs])
        out = ctypes.c_uint64()
        rc = lib().esc_materialize(self.h, table.h, pred.h, pj.ctypes.data if len(pj) else None, len(pj),
                                   ctypes.c_void_p(rowids.data_ptr()) if rowids is not None else None,
                                   optrs, int(capacity), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                   _stream_handle(stream), ctypes.byref(out))
        if rc == ERR_CAPACITY and allow_overflow:
            return out.value
        check(rc)
        return out.value

    def count_conjuncts(self, table: Table, pred: Pred, stream=None):
        """(conjunct counts, prefix counts) of the root AND's children, from
        one scan."""
        cc = np.zeros(MAX_CONJ, np.uint64)
        pc = np.zeros(MAX_CONJ, np.uint64)
        m = ctypes.c_int()
        ws = self.workspace(table, WS_CONJUNCTS, key="conjuncts")
        check(lib().esc_count_conjuncts(self.h, table.h, pred.h, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                        _stream_handle(stream), MAX_CONJ, cc.ctypes.data, pc.ctypes.data,
                                        ctypes.byref(m)))
        return cc[:m.value].tolist(), pc[:m.value].tolist()

    def materialize_async(self, table: Table, pred: Pred, proj, rowids, outs, capacity, dev_count, ws, stream=None):
        """Enqueues the materialization; the full count goes to the device
        tensor dev_count (one int64) in stream order."""
        pj = np.asarray(proj, np.int32)
        optrs = (ctypes.c_void_p * max(len(outs), 1))(*[o.data_ptr() for o in outs])
        check(lib().esc_materialize_async(self.h, table.h, pred.h, pj.ctypes.data if len(pj) else None, len(pj),
                                          ctypes.c_void_p(rowids.data_ptr()) if rowids is not None else None,
                                          optrs, int(capacity), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                          _stream_handle(stream), ctypes.c_void_p(dev_count.data_ptr())))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_ctx_destroy(self.h)
            self.h = None


def device_table(t, device="cuda:0"):
    """Table descriptor over device copies of a datagen.Table's columns."""
    import torch
    cols = []
    for c in t.cols:
        if isinstance(c, np.ndarray):
            c = torch.from_numpy(np.ascontiguousarray(c))
        cols.append(c.to(device).contiguous())
    return Table(t.nrows, t.dtypes, cols)


def schema_table(t):
    return Table(t.nrows, t.dtypes, None)


class Batch:
    """Batched COUNT(*) of many predicates over several tables (one hipGraph
    launch of a persistent kernel).  Its device workspace is a torch tensor
    owned here; an update whose plan no longer fits it re-creates the batch
    on a larger one."""

    def __init__(self, ctx: Context, tables, preds, owner, autotune=False, rows_per_thread=0, group=0,
                 chunk_rows=0, blocks_per_cu=0, max_preds=0, max_cols=0, stream=None):
        self.ctx = ctx
        self.tables = list(tables)
        self._o = BatchOpts(1 if autotune else 0, 0, rows_per_thread, group, chunk_rows, blocks_per_cu,
                            max_preds, max_cols)
        self.h = None
        self._create(preds, owner, stream)

    def _create(self, preds, owner, stream, headroom=1.0):
        import torch
        self.preds = list(preds)
        self.owner = np.ascontiguousarray(owner, np.int32)
        th = (ctypes.c_void_p * len(self.tables))(*[t.h for t in self.tables])
        ph = (ctypes.c_void_p * len(self.preds))(*[p.h for p in self.preds])
        nb = ctypes.c_size_t()
        check(lib().esc_batch_workspace_size(self.ctx.h, th, len(self.tables), ph, self.owner.ctypes.data,
                                             len(self.preds), ctypes.byref(self._o), ctypes.byref(nb)))
        self.ws = torch.empty(int(nb.value * headroom) + 256, dtype=torch.uint8, device=f"cuda:{self.ctx.device}")
        h = ctypes.c_void_p()
        check(lib().esc_batch_create(self.ctx.h, th, len(self.tables), ph, self.owner.ctypes.data, len(self.preds),
                                     ctypes.byref(self._o), ctypes.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                     _stream_handle(stream), ctypes.byref(h)))
        self.h = h

    def count(self, stream=None):
        out = np.zeros(len(self.preds), np.uint64)
        check(lib().esc_batch_count(self.h, _stream_handle(stream), out.ctypes.data))
        return out

    def update(self, preds, owner=None, stream=None):
        owner = self.owner if owner is None else np.ascontiguousarray(owner, np.int32)
        ph = (ctypes.c_void_p * len(preds))(*[p.h for p in preds])
        rc = lib().esc_batch_update(self.h, ph, owner.ctypes.data, len(preds), _stream_handle(stream))
        if rc == ERR_OOM:
            # more predicates or work items than the workspace holds: a new
            # batch (same options; a tuned choice stays cached) on a larger one
            lib().esc_batch_destroy(self.h)
            self.h = None
            self._create(preds, owner, stream, headroom=1.5)
            return
        check(rc)
        self.preds = list(preds)
        self.owner = owner

    def opts(self):
        o = BatchOpts()
        check(lib().esc_batch_get_opts(self.h, ctypes.byref(o)))
        return {"rows_per_thread": o.rows_per_thread, "group": o.group, "chunk_rows": o.chunk_rows,
                "blocks_per_cu": o.blocks_per_cu, "max_cols": o.max_cols}

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_batch_destroy(self.h)
            self.h = None


# ------------------------------------------------------------------ learned gate

def _catalog_args(schema: Table, cmin, cmax, sample):
    nc = min(len(schema.dtypes), 6)
    vmin = (Value * len(schema.dtypes))()
    vmax = (Value * len(schema.dtypes))()

    def put(arr, i, dt, v):
        if dt == FLOAT32:
            arr[i].f = float(np.float32(v))
        else:
            arr[i].i = int(v)

    for c, dt in enumerate(schema.dtypes):
        put(vmin, c, dt, cmin[c])
        put(vmax, c, dt, cmax[c])
    m = 0 if sample is None else len(sample[0])
    vs = (Value * max(nc * m, 1))()
    for c in range(nc if m else 0):
        col = np.asarray(sample[c])
        if len(col) != m:
            raise ValueError("every column sample needs the same length")
        if schema.dtypes[c] == FLOAT32:
            bits = col.astype(np.float32).view(np.uint32)
        else:
            bits = col.astype(np.int64).astype(np.int32).view(np.uint32)
        ctypes.memmove(ctypes.addressof(vs) + c * m * 4, bits.ctypes.data, m * 4)
    return vmin, vmax, vs, m


def featurize(schema: Table, preds, cmin, cmax, sample=None):
    """64 float32 features per compiled predicate (host, in the library).
    sample: per column c < min(ncols, 6), the same number of row values (or
    None: no sample)."""
    vmin, vmax, vs, m = _catalog_args(schema, cmin, cmax, sample)
    ph = (ctypes.c_void_p * max(len(preds), 1))(*[p.h for p in preds])
    out = np.zeros((len(preds), 64), np.float32)
    check(lib().esc_featurize(schema.h, vmin, vmax, vs, m, ph, len(preds), out.ctypes.data))
    return out


class Catalog:
    """A table's catalog in the library (column CDFs built once)."""

    def __init__(self, schema: Table, cmin, cmax, sample=None):
        vmin, vmax, vs, m = _catalog_args(schema, cmin, cmax, sample)
        h = ctypes.c_void_p()
        check(lib().esc_catalog_create(schema.h, vmin, vmax, vs, m, ctypes.byref(h)))
        self.h = h

    def featurize(self, preds):
        ph = (ctypes.c_void_p * max(len(preds), 1))(*[p.h for p in preds])
        out = np.zeros((len(preds), 64), np.float32)
        check(lib().esc_featurize_catalog(self.h, ph, len(preds), out.ctypes.data))
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_catalog_destroy(self.h)
            self.h = None


def params_to_flat(params):
    parts = []
    for w, b in params:
        parts.append(np.asarray(w, np.float32).reshape(-1))
        parts.append(np.asarray(b, np.float32).reshape(-1))
    flat = np.concatenate(parts).astype(np.float32)
    assert flat.size == MLP_NPARAMS
    return flat


def flat_to_params(flat, dims=(64, 256, 256, 256, 1)):
    out, o = [], 0
    for i in range(len(dims) - 1):
        w = flat[o:o + dims[i] * dims[i + 1]].reshape(dims[i], dims[i + 1]); o += w.size
        b = flat[o:o + dims[i + 1]]; o += b.size
        out.append((w, b))
    return out


class MLP:
    """The estimator on the device.  Its state (weights, Adam moments, step
    count, bf16 weight copies) and the training workspace are torch device
    tensors owned here and handed to the library."""

    def __init__(self, ctx: Context, params=None):
        import torch
        self.ctx = ctx
        dev = f"cuda:{ctx.device}"
        self.state = torch.zeros(lib().esc_mlp_state_bytes(), dtype=torch.uint8, device=dev)
        self._ws = None
        h = ctypes.c_void_p()
        check(lib().esc_mlp_create(ctx.h, ctypes.c_void_p(self.state.data_ptr()), self.state.numel(),
                                   ctypes.byref(h)))
        self.h = h
        if params is not None:
            self.set_params(params)

    def workspace(self, batch):
        import torch
        nb = lib().esc_mlp_workspace_bytes(int(batch))
        if nb == 0:
            raise EscError(ERR_INVALID, f"batch {batch} outside [1, 4096]")
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=self.state.device)
        return self._ws

    def set_params(self, params):
        flat = params if isinstance(params, np.ndarray) else params_to_flat(params)
        flat = np.ascontiguousarray(flat, np.float32)
        check(lib().esc_mlp_set_params(self.h, flat.ctypes.data))

    def get_params(self):
        flat = np.zeros(MLP_NPARAMS, np.float32)
        check(lib().esc_mlp_get_params(self.h, flat.ctypes.data))
        return flat

    def get_state(self):
        """(params, adam_m, adam_v, steps)"""
        p, m, v = (np.zeros(MLP_NPARAMS, np.float32) for _ in range(3))
        st = ctypes.c_int64()
        check(lib().esc_mlp_get_state(self.h, p.ctypes.data, m.ctypes.data, v.ctypes.data, ctypes.byref(st)))
        return p, m, v, st.value

    def set_state(self, params, adam_m, adam_v, steps):
        arrs = [np.ascontiguousarray(a, np.float32) for a in (params, adam_m, adam_v)]
        check(lib().esc_mlp_set_state(self.h, arrs[0].ctypes.data, arrs[1].ctypes.data, arrs[2].ctypes.data,
                                      int(steps)))

    def save(self, path):
        check(lib().esc_mlp_save(self.h, os.fsencode(path)))

    def load(self, path):
        check(lib().esc_mlp_load(self.h, os.fsencode(path)))

    def predict(self, x, out=None, stream=None):
        import torch
        n = x.shape[0]
        out = torch.empty(n, dtype=torch.float32, device=x.device) if out is None else out
        check(lib().esc_mlp_predict(self.h, ctypes.c_void_p(x.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                    _stream_handle(stream)))
        return out

    def gradients(self, x, y, stream=None):
        import torch
        g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=x.device)
        ws = self.workspace(x.shape[0])
        check(lib().esc_mlp_gradients(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      x.shape[0], ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel(), _stream_handle(stream)))
        return g

    def train(self, x, y, order, steps, batch, lr=1e-3, stream=None, want_loss=True):
        import torch
        loss = torch.zeros(max(steps, 1), dtype=torch.float32, device=x.device) if want_loss else None
        ws = self.workspace(batch)
        check(lib().esc_mlp_train(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(order.data_ptr()), steps, batch, float(lr),
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(stream),
                                  ctypes.c_void_p(loss.data_ptr()) if want_loss else None))
        return loss[:steps].cpu().numpy() if want_loss else np.zeros(0, np.float32)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.esc_mlp_destroy(self.h)
            self.h = None


def gate_pushdown(yhat, nrows, tau, beta, min_rows):
    y = np.ascontiguousarray(yhat, np.float32)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(nrows, np.int64), y.shape))
    r = np.zeros(len(y), np.uint8)
    check(lib().esc_gate_pushdown(y.ctypes.data, n.ctypes.data, len(y), tau, beta, int(min_rows), r.ctypes.data))
    return r.astype(bool)


def gate_join_pair(yr, nr, ys, ns, beta):
    r = ctypes.c_uint8()
    check(lib().esc_gate_join_pair(float(yr), int(nr), float(ys), int(ns), float(beta), ctypes.byref(r)))
    return bool(r.value)


def gate_join_pairs(yr, nr, ys, ns, beta, tie_sel=0.0):
    """esc_gate_join_pairs: one route per query (ties: tie_sel)."""
    a = np.ascontiguousarray(yr, np.float32)
    b = np.ascontiguousarray(ys, np.float32)
    if a.shape != b.shape:
        raise ValueError("yr and ys differ in length")
    r = np.zeros(len(a), np.uint8)
    check(lib().esc_gate_join_pairs(a.ctypes.data, int(nr), b.ctypes.data, int(ns), len(a), float(beta),
                                    float(tie_sel), r.ctypes.data))
    return r.astype(bool)


def policy_keep(model: CostModel, nrows, counts, scan_cols, proj_cols, reuses=1):
    """Materialize-or-not for each selection; returns (keep, saving_s)."""
    c = np.ascontiguousarray(counts, np.uint64)
    n = np.ascontiguousarray(np.broadcast_to(np.asarray(nrows, np.int64), c.shape))
    keep = np.zeros(len(c), np.uint8)
    saving = np.zeros(len(c), np.float64)
    check(lib().esc_policy_keep(ctypes.byref(model), n.ctypes.data, c.ctypes.data, len(c), int(scan_cols),
                                int(proj_cols), int(reuses), keep.ctypes.data, saving.ctypes.data))
    return keep.astype(bool), saving


def policy_thresholds(model: CostModel, nrows, scan_cols, proj_cols, reuses=1):
    """(tau, min_rows) implied by the model for a table shape."""
    tau, mr = ctypes.c_double(), ctypes.c_double()
    check(lib().esc_policy_thresholds(ctypes.byref(model), int(nrows), int(scan_cols), int(proj_cols), int(reuses),
                                      ctypes.byref(tau), ctypes.byref(mr)))
    return tau.value, mr.value
