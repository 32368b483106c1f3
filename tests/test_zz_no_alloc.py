"""The allocation-free materialization (esc_materialize_noalloc, workspace
in the library's static device array) against esc_materialize_async on a
caller-owned workspace: same count, row ids and projected values, on two
calls in a row, the second on a smaller table, and through the C ABI."""
import ctypes

import numpy as np
import pytest

from oracle import scan
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def _outputs(n, proj, dt):
    import torch
    ids = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    outs = [torch.full((n,), -7, dtype=torch.int32, device="cuda").view(dt.cols[j].dtype) for j in proj]
    return ids, outs


def _noalloc(ctx, dt, p, proj, ids, outs, capacity):
    import torch
    dev_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    pc = (ctypes.c_int32 * len(proj))(*proj)
    po = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
    rc = esc.lib().esc_materialize_noalloc(ctx.h, dt.h, p.h, pc, len(proj), ctypes.c_void_p(ids.data_ptr()), po,
                                           capacity, None, ctypes.c_void_p(dev_count.data_ptr()))
    torch.cuda.synchronize()
    return rc, int(dev_count.item())


def _async(ctx, dt, p, proj, ids, outs, capacity):
    import torch
    dev_count = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.zeros(ctx.workspace(dt, True, key="noalloc-size").numel(), dtype=torch.uint8, device="cuda")
    ctx.materialize_async(dt, p, proj, ids, outs, capacity, dev_count, ws=ws)
    torch.cuda.synchronize()
    return int(dev_count.item())


def test_noalloc_matches_async_two_calls(ctx):
    proj = dg.PLAIN_PROJECTION
    prev = None
    for n, seed in ((1_000_003, 61), (200_001, 62)):   # the second call on a smaller table
        t = dg.table_plain(n, seed=seed)
        dt = esc.device_table(t)
        for spec in (dg.pred_plain(t, 3), ("lt", 2, 250_000)):
            p = esc.Pred(dt, spec)
            ids_a, outs_a = _outputs(n, proj, dt)
            want = _async(ctx, dt, p, proj, ids_a, outs_a, n)
            ids_b, outs_b = _outputs(n, proj, dt)
            rc, got = _noalloc(ctx, dt, p, proj, ids_b, outs_b, n)
            assert rc == esc.OK, esc.last_error()
            assert got == want == scan.count(t, spec)
            # everything written, and nothing past the count
            assert np.array_equal(ids_b.cpu().numpy(), ids_a.cpu().numpy())
            for a, b in zip(outs_a, outs_b):
                assert np.array_equal(b.cpu().numpy().view(np.uint32), a.cpu().numpy().view(np.uint32))
            if prev is not None:
                assert prev != (n, got)
            prev = (n, got)


def test_noalloc_capacity_and_limit(ctx):
    """A capacity below the count writes the first rows and reports the full
    count; a table beyond the static scratch is refused before any launch."""
    import torch
    t = dg.table_plain(300_007, seed=63)
    dt = esc.device_table(t)
    spec = ("lt", 2, 500_000)
    p = esc.Pred(dt, spec)
    wc, wids, wouts = scan.materialize(t, spec, dg.PLAIN_PROJECTION)
    cap = wc // 2
    ids, outs = _outputs(max(cap, 1), dg.PLAIN_PROJECTION, dt)
    rc, got = _noalloc(ctx, dt, p, dg.PLAIN_PROJECTION, ids, outs, cap)
    assert rc == esc.OK and got == wc
    assert np.array_equal(ids[:cap].cpu().numpy(), wids[:cap])
    # 131M rows of a real (zero-filled) device column: one-column programs need
    # more than the 16 MiB array
    big = torch.zeros(131_000_000, dtype=torch.int32, device="cuda")
    bt = esc.Table(big.numel(), [dg.INT32], [big])
    bp = esc.Pred(bt, ("lt", 0, 5))
    ids1, outs1 = _outputs(1, [0], bt)
    rc, _ = _noalloc(ctx, bt, bp, [0], ids1, outs1, 1)
    assert rc == esc.ERR_CAPACITY
    assert "static scratch" in esc.last_error()
