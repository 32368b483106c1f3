"""Materialization policy with thresholds from measured costs.

Section 2.1 materializes a pushed-down selection only when it prunes enough
rows and the table is large enough, with both limits left to the DBA and
adaptive choices named as future work.  `calibrate` measures the cost
model of libesc's policy (esc_policy_keep / esc_policy_thresholds) on the
device with the library's own kernels:
  scan_bytes_per_s  back-to-back counts whose predicate reads every column
                    of a re-read (the cost of re-reading the table);
  fixed_s           the materialization time of an empty selection (count
                    already done, so only the offsets and the write pass run);
  sparse_row_s      a least-squares line through the materialization times
                    of `lt k` selections on the permutation key below the
                    dense fraction (projected values gathered);
  dense_bytes_per_s, dense_row_s
                    a line through those above it (projected columns read
                    whole: the intercept is the column read);
  tmp_bytes_per_s   counts over the temporary table of the largest of them
                    (row ids and projected columns).
Every count and materialization runs inside libesc; this module only
times them (HIP events through torch) and fits the line.
"""
from __future__ import annotations

import numpy as np

from . import esc


def _touch_all(ncols):
    """A predicate that reads columns 0..ncols-1 (non-negative int columns) and is not folded."""
    leaves = [("gt", c, -1) for c in range(ncols)]
    return ("and", leaves) if ncols > 1 else leaves[0]


def _time_ms(torch, fn, reps, evict=None):
    """Median milliseconds of fn() over reps runs, each after `evict`."""
    out = []
    for _ in range(reps):
        if evict is not None:
            evict()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def calibrate(ctx, table: esc.Table, key_col, proj, scan_cols,
              sparse_fractions=(1e-4, 1e-3, 4e-3), dense_fractions=(0.02, 0.1, 0.3, 0.6), reps=5):
    """Cost model for materializing `proj` (projected column indices) of
    selections on `table`, whose column key_col holds a permutation of
    0..nrows-1 and whose first scan_cols columns are non-negative ints.
    `lt k` selections on the key spread their rows evenly, so a selectivity
    below the dense fraction gathers projected values row by row and one
    above it reads the projected columns whole.  Returns (esc.CostModel,
    details)."""
    import torch
    dev = table.cols[0].device
    n = table.nrows
    scratch = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB: evicts the caches
    evict = lambda: scratch.sum()
    # re-read of the table: every scanned column streamed once
    p_all = esc.Pred(table, _touch_all(scan_cols))
    ws_c = ctx.workspace(table, False, key=("policy", "scan"))
    dcnt = torch.zeros(1, dtype=torch.int64, device=dev)
    ms_scan = _time_ms(torch, lambda: ctx.count_async(table, p_all, dcnt, ws_c), reps, evict)
    scan_rate = n * 4.0 * scan_cols / (ms_scan * 1e-3)
    # materialization after the decision's count (offsets and write pass)
    dense_fraction = ctx.dense_fraction()
    ks_sparse = [int(f * n) for f in sparse_fractions if f < dense_fraction]
    ks_dense = [int(f * n) for f in dense_fractions if f >= dense_fraction]
    ks = [0] + ks_sparse + ks_dense
    cap = max(max(ks), 1)
    ws_m = ctx.workspace(table, True, key=("policy", "mat"))
    rowids = torch.empty(cap, dtype=torch.int32, device=dev)
    outs = [torch.empty(cap, dtype=table.cols[j].dtype, device=dev) for j in proj]
    dmat = torch.zeros(1, dtype=torch.int64, device=dev)
    ms_mat = {}
    for k in ks:
        p = esc.Pred(table, ("lt", key_col, k))
        times = []
        for _ in range(reps):
            ctx.count(table, p, ws=ws_m)          # the count the decision needs; leaves tile masks
            evict()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            ctx.materialize_async(table, p, proj, rowids, outs, cap, dmat, ws_m)
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
        assert int(dmat.item()) == k
        ms_mat[k] = float(np.median(times))
    fixed_ms = ms_mat[0]
    xs = np.asarray(ks_sparse, np.float64)
    ys = np.asarray([ms_mat[k] for k in ks_sparse]) - fixed_ms
    sparse_row_ms = float(xs @ ys / (xs @ xs)) if len(xs) else 0.0
    A = np.stack([np.ones(len(ks_dense)), np.asarray(ks_dense, np.float64)], axis=1)
    (cols_ms, dense_row_ms), *_ = np.linalg.lstsq(A, np.asarray([ms_mat[k] for k in ks_dense]) - fixed_ms,
                                                   rcond=None)
    col_bytes = n * 4.0 * len(proj)
    dense_rate = col_bytes / (cols_ms * 1e-3) if col_bytes > 0 and cols_ms > 0 else 1e15
    # reading the temporary table of the largest selection
    kmax = max(ks)
    tmp = esc.Table(kmax, [esc.INT32] + [table.dtypes[j] for j in proj], [rowids[:kmax]] + [o[:kmax] for o in outs])
    ncols_tmp = 1 + len(proj)
    ints = all(table.dtypes[j] != esc.FLOAT32 for j in proj)
    p_tmp = esc.Pred(tmp, _touch_all(ncols_tmp if ints else 1))
    ws_t = ctx.workspace(tmp, False, key=("policy", "tmp"))
    ms_tmp = _time_ms(torch, lambda: ctx.count_async(tmp, p_tmp, dcnt, ws_t), reps, evict)
    tmp_rate = kmax * 4.0 * (ncols_tmp if ints else 1) / (ms_tmp * 1e-3)
    m = esc.CostModel(scan_rate, max(fixed_ms, 0.0) * 1e-3, max(sparse_row_ms, 0.0) * 1e-3, dense_fraction,
                      dense_rate, max(float(dense_row_ms), 0.0) * 1e-3, tmp_rate)
    details = {"scan_ms": ms_scan, "mat_ms": ms_mat, "tmp_ms": ms_tmp, "tmp_rows": kmax,
               "fit_fixed_ms": fixed_ms, "fit_sparse_row_ns": sparse_row_ms * 1e6,
               "fit_dense_cols_ms": float(cols_ms), "fit_dense_row_ns": float(dense_row_ms) * 1e6}
    return m, details


def model_dict(m: esc.CostModel):
    return {name: getattr(m, name) for name, _ in m._fields_}
