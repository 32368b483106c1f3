"""GPU parity of esc_count / esc_materialize against the CPU oracle.

Counts, row ids and projected values must be bit-exact: every comparison is
exact in the column's dtype, and row order is ascending row index."""
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


def gpu_materialize(ctx, dt, pred, proj, capacity=None):
    import torch
    p = esc.Pred(dt, pred)
    n = ctx.count(dt, p)
    cap = n if capacity is None else capacity
    rowids = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    outs = [torch.zeros(max(cap, 1), dtype=dt.cols[j].dtype, device="cuda") for j in proj]
    c = ctx.materialize(dt, p, proj, rowids, outs, cap, allow_overflow=capacity is not None)
    k = min(c, cap)
    return n, c, rowids[:k].cpu().numpy(), [o[:k].cpu().numpy() for o in outs]


def assert_same_rows(got_ids, got_outs, want_ids, want_outs):
    assert np.array_equal(got_ids, want_ids)
    for g, w in zip(got_outs, want_outs):
        assert np.array_equal(g.view(np.uint32), w.view(np.uint32))


# wave tiles are 64*RPT rows (RPT 8, 16 or 32): cover empty, ragged and multi-tile inputs
SIZES = [0, 1, 3, 4, 5, 63, 64, 65, 1023, 1024, 1025, 2047, 2048, 2049, 4097, 20_001]


@pytest.mark.parametrize("n", SIZES)
def test_random_trees_small_tables(ctx, n):
    rng = np.random.default_rng(500 + n)
    cols = [rng.integers(-5, 6, n).astype(np.int32),
            rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32),
            rng.choice(np.array([0.0, -0.0, 1.0, -1.0, 2.5, np.inf, -np.inf, np.nan, 1e-45, -1e-45], np.float32), n),
            rng.integers(0, 4, n).astype(np.int32)]
    t = dg.Table("tiny", n, [dg.INT32, dg.INT32, dg.FLOAT32, dg.DATE32], cols, ["u"] * 4, [None] * 4)
    dt = esc.device_table(t)
    for i in range(40):
        p = dg.random_pred_tiny(t, rng)
        want = scan.count(t, p)
        try:
            n_gpu, c, ids, outs = gpu_materialize(ctx, dt, p, [2, 0, 3])
        except esc.EscError as e:   # deep random trees may exceed the compiled limits
            assert e.status == esc.ERR_UNSUPPORTED, (e, scan.to_sexpr(p, t.dtypes))
            continue
        assert n_gpu == want == c, scan.to_sexpr(p, t.dtypes)
        wc, wids, wouts = scan.materialize(t, p, [2, 0, 3])
        assert_same_rows(ids, outs, wids, wouts)


@pytest.mark.parametrize("k", [5, 6, 7, 8])
def test_wide_programs_materialize(ctx, k):
    """Conjunctions over five to eight distinct columns, with and without a
    udf leaf: the counts that store tiles for the materialization run 32 rows
    per lane up to six columns and 16 above; counts, row ids and projected
    values equal the oracle's (150,001 rows: many tiles and a ragged one)."""
    rng = np.random.default_rng(900 + k)
    n = 150_001
    cols = [rng.integers(0, 100, n).astype(np.int32) for _ in range(8)]
    t = dg.Table("wide", n, [dg.INT32] * 8, cols, ["u"] * 8, [None] * 8)
    dt = esc.device_table(t)
    for trial in range(4):
        cs = [int(c) for c in rng.choice(8, k, replace=False)]
        leaves = [("lt", c, int(rng.integers(55, 100))) for c in cs]
        if trial % 2:
            leaves[0] = ("udf", ("add", ("col", cs[0]), ("col", cs[1])), ("lt", int(rng.integers(90, 170))))
        p = ("and", leaves)
        want = scan.count(t, p)
        assert want > 0
        proj = [cs[0], cs[-1]]
        n_gpu, c, ids, outs = gpu_materialize(ctx, dt, p, proj)
        assert n_gpu == c == want, scan.to_sexpr(p, t.dtypes)
        wc, wids, wouts = scan.materialize(t, p, proj)
        assert_same_rows(ids, outs, wids, wouts)


def test_edge_values(ctx):
    from test_oracle_scan import EDGE_CASES, edge_pred
    t = dg.table_edge_floats()
    dt = esc.device_table(t)
    for pred, want in EDGE_CASES:
        pred = edge_pred(pred, t)
        assert ctx.count(dt, esc.Pred(dt, pred)) == want == scan.count(t, pred), pred


def test_plain_config_100_seeds(ctx):
    """The Section 1 selection on R(A,B,C,D) with 1M rows, 100 constant draws:
    count, then row ids with the projection A, C, D in row order."""
    t = dg.table_plain(1_000_000)
    dt = esc.device_table(t)
    total = 0
    for s in range(100):
        p = dg.pred_plain(t, s)
        n, c, ids, outs = gpu_materialize(ctx, dt, p, dg.PLAIN_PROJECTION)
        wc, wids, wouts = scan.materialize(t, p, dg.PLAIN_PROJECTION)
        assert n == c == wc, s
        assert_same_rows(ids, outs, wids, wouts)
        total += n
    assert total > 0


def test_closed_forms_on_gpu(ctx):
    n = 3_000_001
    t = dg.table_plain(n, seed=77)
    dt = esc.device_table(t)
    for k in [0, 1, 2047, 2048, 2049, 1_500_000, n - 1, n]:
        assert ctx.count(dt, esc.Pred(dt, ("lt", 0, k))) == k
    for a, b in [(0, 0), (10, 5000), (0, n - 1), (n - 100, n + 100)]:
        assert ctx.count(dt, esc.Pred(dt, ("between", 0, a, b))) == min(b, n - 1) - a + 1
    assert sum(ctx.count(dt, esc.Pred(dt, ("udf", dg.UDF_PLAIN, ("eq", w)))) for w in range(97)) == n
    # everything qualifies: row ids are 0..n-1 and the projection is the column itself
    import torch
    p = esc.Pred(dt, ("gt", 0, -1))
    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    assert ctx.materialize(dt, p, [1], ids, [out], n) == n
    assert torch.equal(ids.cpu(), torch.arange(n, dtype=torch.int32))
    assert torch.equal(out, dt.cols[1])


def test_capacity_overflow(ctx):
    t = dg.table_plain(100_000, seed=78)
    dt = esc.device_table(t)
    p = ("lt", 0, 5000)
    n, c, ids, (a,) = gpu_materialize(ctx, dt, p, [0], capacity=4321)
    assert n == c == 5000 and len(ids) == 4321
    wc, wids, (wa,) = scan.materialize(t, p, [0], capacity=4321)
    assert np.array_equal(ids, wids) and np.array_equal(a, wa)
    import torch
    pr = esc.Pred(dt, p)
    ids = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(esc.EscError) as e:
        ctx.materialize(dt, pr, [], ids, [], 1)
    assert e.value.status == esc.ERR_CAPACITY


def test_determinism_repeat(ctx):
    import torch
    t = dg.table_star(2_000_000, seed=79)
    dt = esc.device_table(t)
    p = esc.Pred(dt, dg.preds_star(t, 4, seed=80)[3])
    n = ctx.count(dt, p)
    ids0 = None
    for _ in range(30):
        ids = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        outs = [torch.empty(max(n, 1), dtype=torch.int32, device="cuda")]
        assert ctx.materialize(dt, p, [6], ids, outs, n) == n
        if ids0 is None:
            ids0 = ids.clone()
        assert torch.equal(ids, ids0)


def test_star_reduced_all_predicates(ctx):
    t = dg.table_star(3_000_000, seed=81)
    dt = esc.device_table(t)
    for i, p in enumerate(dg.preds_star(t, 32, seed=82)):
        n, c, ids, outs = gpu_materialize(ctx, dt, p, dg.STAR_PROJECTION)
        wc, wids, wouts = scan.materialize(t, p, dg.STAR_PROJECTION)
        assert n == c == wc, i
        assert_same_rows(ids, outs, wids, wouts)


def test_star_full_size_counts_and_rows(ctx):
    """60M-row star table, 32 predicates, in the launch configuration the
    benchmark times (count, then materialize on the count's workspace): every
    count, row id and projected value against the oracle (run in threads:
    the C oracle releases the interpreter lock)."""
    import concurrent.futures as cf

    import torch
    td = dg.table_star(device="cuda")      # the benchmark's table, drawn on the device
    preds = dg.preds_star(td, 32)
    dt = esc.Table(td.nrows, td.dtypes, td.cols)
    t = td.host()
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        want = list(ex.map(lambda p: scan.materialize(t, p, dg.STAR_PROJECTION), preds))
    for i, p in enumerate(preds):
        pr = esc.Pred(dt, p)
        n = ctx.count(dt, pr)
        wc, wids, wouts = want[i]
        assert n == wc, i
        ids = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
        outs = [torch.empty(max(n, 1), dtype=dt.cols[j].dtype, device="cuda") for j in dg.STAR_PROJECTION]
        assert ctx.materialize(dt, pr, dg.STAR_PROJECTION, ids, outs, n) == n
        assert_same_rows(ids[:n].cpu().numpy(), [o[:n].cpu().numpy() for o in outs], wids, wouts)


def test_offset_scan_over_several_rounds(ctx):
    """The offset scan runs in rounds of 16384 wave tiles with a carry
    between them: a one-column table of 2^26 + 12345 rows has 32775 tiles of
    2048 rows, so its materialization takes three rounds (the last one
    ragged, as is the last tile); row ids and values equal the oracle's, for
    a dense and a sparse selection."""
    rng = np.random.default_rng(515)
    n = (1 << 26) + 12_345
    col = rng.integers(0, 1000, n, dtype=np.int32)
    t = dg.Table("rounds", n, [dg.INT32], [col], ["u"], [None])
    dt = esc.device_table(t)
    for pred in (("lt", 0, 500), ("eq", 0, 7)):
        want = scan.count(t, pred)
        got, c, ids, outs = gpu_materialize(ctx, dt, pred, [0])
        assert got == c == want, pred
        wc, wids, wouts = scan.materialize(t, pred, [0])
        assert wc == want
        assert_same_rows(ids, outs, wids, wouts)


def test_constant_predicates_materialize(ctx):
    """Always-true and always-false predicates (folded at compile time) still
    materialize every / no row, also on a fresh workspace."""
    import torch
    t = dg.table_plain(5_000, seed=83)
    dt = esc.device_table(t)
    for spec, want in [(("between", 1, -2**31, 2**31 - 1), t.nrows), (("lt", 1, -2**31), 0)]:
        p = esc.Pred(dt, spec)
        assert p.info()["constant"] != 0
        ids = torch.full((t.nrows,), -1, dtype=torch.int32, device="cuda")
        out = torch.zeros(t.nrows, dtype=torch.int32, device="cuda")
        ws = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
        assert ctx.materialize(dt, p, [2], ids, [out], t.nrows, ws=ws) == want
        assert ctx.count(dt, p, ws=ws) == want
        if want:
            assert torch.equal(ids.cpu(), torch.arange(t.nrows, dtype=torch.int32))
            assert torch.equal(out, dt.cols[2])


def test_materialize_reuse_and_density_mix(ctx):
    """The write pass reads the truth masks the count pass left in the
    workspace.  On one workspace: materialize after the same predicate's
    count (masks reused), after another predicate's count (must count
    again), and twice in a row; predicates whose tiles are dense (coalesced
    projection loads), sparse (gathers), mixed, and near the switch-over
    density of 1 in 16.  Rows and projections against the oracle."""
    import torch
    n = 1_000_003
    rng = np.random.default_rng(91)
    cols = [np.arange(n, dtype=np.int32),
            rng.integers(0, 4096, n).astype(np.int32),
            rng.standard_normal(n).astype(np.float32)]
    t = dg.Table("mix", n, [dg.INT32, dg.INT32, dg.FLOAT32], cols, ["u"] * 3, [None] * 3)
    dt = esc.device_table(t)
    specs = {
        "dense_block": ("between", 0, n // 3, n // 2),
        "sparse": ("eq", 1, 7),
        "mixed": ("or", [("between", 0, 100_000, 180_000), ("eq", 1, 9)]),
        "near_16th": ("lt", 1, 256),
        "float": ("and", [("gt", 2, 0.5), ("lt", 1, 3000)]),
    }
    preds = {k: esc.Pred(dt, v) for k, v in specs.items()}
    want = {k: scan.materialize(t, v, [2, 1, 0]) for k, v in specs.items()}
    ws = ctx.workspace(dt, True, key="reuse-test")   # the same workspace throughout
    ids = torch.empty(n, dtype=torch.int32, device="cuda")
    outs = [torch.empty(n, dtype=dt.cols[j].dtype, device="cuda") for j in (2, 1, 0)]

    def mat(k):
        c = ctx.materialize(dt, preds[k], [2, 1, 0], ids, outs, n, ws=ws)
        wc, wids, wouts = want[k]
        assert c == wc, k
        assert_same_rows(ids[:c].cpu().numpy(), [o[:c].cpu().numpy() for o in outs], wids, wouts)

    order = ["dense_block", "sparse", "mixed", "near_16th", "float"]
    for k in order:                       # count, then materialize with the masks it left
        assert ctx.count(dt, preds[k], ws=ws) == want[k][0]
        mat(k)
    assert ctx.count(dt, preds["sparse"], ws=ws) == want["sparse"][0]
    mat("dense_block")                    # masks belong to another predicate: counts again
    mat("mixed")
    mat("mixed")                          # twice in a row
    for k in reversed(order):             # materialize without a preceding count
        mat(k)


def test_materialize_through_reused_workspace_address(ctx):
    """A count leaves its tiles in a workspace; the caller frees it and the
    allocator hands the same address out again, zero-filled.  A
    materialization of the same table and predicate on the new
    buffer, with no count before it, must count afresh (the workspace's stamp
    no longer matches) and give the oracle's rows."""
    import torch
    t = dg.table_plain(300_007, seed=95)
    dt = esc.device_table(t)
    spec = ("lt", 2, 400_000)
    p = esc.Pred(dt, spec)
    wc, wids, wouts = scan.materialize(t, spec, dg.PLAIN_PROJECTION)
    assert wc > 0
    size = ctx.workspace(dt, True, key="size-probe").numel()
    ids = torch.empty(t.nrows, dtype=torch.int32, device="cuda")
    outs = [torch.empty(t.nrows, dtype=torch.int32, device="cuda") for _ in dg.PLAIN_PROJECTION]

    def materialize_on(ws):
        # straight through the C ABI: no workspace initialisation by the binding
        cnt = esc.ctypes.c_uint64()
        pc = (esc.ctypes.c_int32 * len(dg.PLAIN_PROJECTION))(*dg.PLAIN_PROJECTION)
        po = (esc.ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        esc.check(esc.lib().esc_materialize(ctx.h, dt.h, p.h, pc, len(outs), esc.ctypes.c_void_p(ids.data_ptr()),
                                            po, t.nrows, esc.ctypes.c_void_p(ws.data_ptr()), ws.numel(), None,
                                            esc.ctypes.byref(cnt)))
        torch.cuda.synchronize()
        assert cnt.value == wc
        assert_same_rows(ids[:wc].cpu().numpy(), [o[:wc].cpu().numpy() for o in outs], wids, wouts)

    ws = torch.zeros(size, dtype=torch.uint8, device="cuda")
    addr = ws.data_ptr()
    assert ctx.count(dt, p, ws=ws) == wc          # tiles stored, stamp written
    materialize_on(ws)                            # reuse on the same workspace
    del ws
    ws2 = torch.zeros(size, dtype=torch.uint8, device="cuda")   # a fresh, zero-filled workspace
    if ws2.data_ptr() != addr:
        pytest.skip("the allocator did not return the freed address")
    materialize_on(ws2)


def test_max_rows_closed_forms(ctx):
    """The largest table the ABI allows (2^31 - 1 rows, row ids are int32):
    A = row index, so count(A < k) = k, a BETWEEN near the end selects known
    rows, and the batched kernel agrees."""
    import torch
    n = 2**31 - 1
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    dt = esc.Table(n, [dg.INT32], [a])
    for k in (0, 1, 12_345_678, n - 5, n):
        assert ctx.count(dt, esc.Pred(dt, ("lt", 0, k))) == k
    assert ctx.count(dt, esc.Pred(dt, ("gt", 0, n - 2))) == 1
    p = esc.Pred(dt, ("between", 0, n - 1000, n - 1))
    ids = torch.empty(1000, dtype=torch.int32, device="cuda")
    out = torch.empty(1000, dtype=torch.int32, device="cuda")
    assert ctx.count(dt, p) == 1000
    assert ctx.materialize(dt, p, [0], ids, [out], 1000) == 1000
    want = torch.arange(n - 1000, n, dtype=torch.int32, device="cuda")
    assert torch.equal(ids, want) and torch.equal(out, want)
    preds = [("lt", 0, 7), ("between", 0, 2**30, 2**30 + 99), ("gt", 0, n - 11), ("eq", 0, n - 1)]
    b = esc.Batch(ctx, [dt], [esc.Pred(dt, q) for q in preds], [0] * len(preds))
    assert b.count().tolist() == [7, 100, 10, 1]
    del b, a, ids, out, want
    torch.cuda.empty_cache()


def test_materialize_async_matches_sync(ctx):
    """esc_materialize_async enqueues the same passes and leaves the count in
    device memory: rows and projections equal the blocking call's, also with
    a capacity below the count (first rows written) and for a constant-false
    predicate."""
    import torch
    t = dg.table_star(1_500_001, seed=93)
    dt = esc.device_table(t)
    specs = dg.preds_star(t, 6, seed=94) + [("lt", 2, -2**31)]
    ws_a = ctx.workspace(dt, True, key="async-a")
    ws_s = ctx.workspace(dt, True, key="async-s")
    dcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    for i, spec in enumerate(specs):
        p = esc.Pred(dt, spec)
        n = scan.count(t, spec)
        for cap in (n, max(n // 3, 1)):
            ids_a = torch.full((max(cap, 1),), -1, dtype=torch.int32, device="cuda")
            outs_a = [torch.zeros(max(cap, 1), dtype=dt.cols[j].dtype, device="cuda") for j in dg.STAR_PROJECTION]
            ids_s = torch.full_like(ids_a, -1)
            outs_s = [torch.zeros_like(o) for o in outs_a]
            if i % 2 == 0:
                assert ctx.count(dt, p, ws=ws_a) == n   # masks reused by the async call
            ctx.materialize_async(dt, p, dg.STAR_PROJECTION, ids_a, outs_a, cap, dcount, ws_a)
            torch.cuda.synchronize()
            assert int(dcount.item()) == n, (i, cap)
            c = ctx.materialize(dt, p, dg.STAR_PROJECTION, ids_s, outs_s, cap, ws=ws_s, allow_overflow=True)
            assert c == n
            k = min(n, cap)
            assert torch.equal(ids_a[:k], ids_s[:k])
            for a, b in zip(outs_a, outs_s):
                assert torch.equal(a[:k].view(torch.int32), b[:k].view(torch.int32))
            if cap < n:
                assert bool((ids_a[k:] == -1).all())


def test_count_begin_end_pipelined(ctx):
    """esc_count_begin / esc_count_end: counts of several selections in
    flight on distinct slots equal the oracle's; a materialization enqueued
    after the next selection's count (the pipelined decide loop, two
    workspaces in turn) reuses its own tiles and equals the blocking call's;
    misuse of a slot is refused."""
    import torch
    t = dg.table_star(1_200_003, seed=95)
    dt = esc.device_table(t)
    specs = dg.preds_star(t, 8, seed=96)
    cps = [esc.Pred(dt, s_) for s_ in specs]
    want = [scan.count(t, s_) for s_ in specs]
    ws = [ctx.workspace(dt, True, key=("pipe", k)) for k in range(2)]
    wsc = ctx.workspace(dt, False, key="pipe-count")
    # three counts in flight, taken out of order
    for k in range(3):
        ctx.count_begin(dt, cps[k], wsc if k == 2 else ws[k], slot=10 + k)
    assert [ctx.count_end(12), ctx.count_end(10), ctx.count_end(11)] == [want[2], want[0], want[1]]
    # the pipelined loop of the star step
    cap = max(want)
    ids = [torch.full((cap,), -1, dtype=torch.int32, device="cuda") for _ in specs]
    outs = [[torch.zeros(cap, dtype=dt.cols[j].dtype, device="cuda") for j in dg.STAR_PROJECTION] for _ in specs]
    dmat = torch.zeros(len(specs), dtype=torch.int64, device="cuda")
    ctx.count_begin(dt, cps[0], ws[0], slot=0)
    got = []
    for i in range(len(specs)):
        if i + 1 < len(specs):
            ctx.count_begin(dt, cps[i + 1], ws[(i + 1) % 2], slot=(i + 1) % 2)
        got.append(ctx.count_end(i % 2))
        ctx.materialize_async(dt, cps[i], dg.STAR_PROJECTION, ids[i], outs[i], cap, dmat[i:i + 1], ws[i % 2])
    torch.cuda.synchronize()
    assert got == want and dmat.cpu().tolist() == want
    for i, s_ in enumerate(specs):
        _, wids, wouts = scan.materialize(t, s_, dg.STAR_PROJECTION)
        assert_same_rows(ids[i][:want[i]].cpu().numpy(), [o[:want[i]].cpu().numpy() for o in outs[i]], wids, wouts)
    # misuse: a slot whose count was not taken, a slot with nothing in flight
    ctx.count_begin(dt, cps[0], wsc, slot=5)
    with pytest.raises(esc.EscError):
        ctx.count_begin(dt, cps[1], wsc, slot=5)
    assert ctx.count_end(5) == want[0]
    with pytest.raises(esc.EscError):
        ctx.count_end(5)
    with pytest.raises(esc.EscError):
        ctx.count_begin(dt, cps[0], wsc, slot=64)


def test_graph_capture_replay(ctx):
    """esc_count_async and esc_materialize_async enqueue kernels only (no
    memset or host copy), so they can be captured into a HIP graph; every
    replay, with eager work and synchronisations between replays, gives the
    exact count and rows."""
    import torch
    t = dg.table_star(1_000_003, seed=98)
    dt = esc.device_table(t)
    spec = dg.preds_star(t, 4, seed=99)[2]
    p = esc.Pred(dt, spec)
    want_n, want_ids, want_outs = scan.materialize(t, spec, [6])
    ws_c = ctx.workspace(dt, False, key="graph-count")
    ws_m = ctx.workspace(dt, True, key="graph-mat")
    dcount = torch.zeros(1, dtype=torch.int64, device="cuda")
    dmat = torch.zeros(1, dtype=torch.int64, device="cuda")
    ids = torch.empty(max(want_n, 1), dtype=torch.int32, device="cuda")
    out = torch.empty(max(want_n, 1), dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):   # warm-up on the capture stream
        ctx.count_async(dt, p, dcount, ws_c, stream=s)
        ctx.materialize_async(dt, p, [6], ids, [out], want_n, dmat, ws_m, stream=s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ctx.count_async(dt, p, dcount, ws_c, stream=s)
        ctx.materialize_async(dt, p, [6], ids, [out], want_n, dmat, ws_m, stream=s)
    for r in range(5):
        dcount.zero_()
        dmat.zero_()
        ids.fill_(-1)
        torch.zeros(1 << 20, device="cuda").add_(1)   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(dcount.item()) == want_n and int(dmat.item()) == want_n, r
        assert np.array_equal(ids[:want_n].cpu().numpy(), want_ids), r
        assert np.array_equal(out[:want_n].cpu().numpy().view(np.uint32), want_outs[0].view(np.uint32)), r


def test_in_slot_tables(ctx, monkeypatch):
    """IN-lists compiled to slot tables count exactly what the oracle counts,
    and what the compare-list form counts, on data built to hit the table
    slots of the keys with other values (keys with one bit flipped), on
    float lists holding zeros, NaN and infinities, on 3..64-key lists, and on
    lists that only a multiplicative slot hash separates."""
    rng = np.random.default_rng(4242)
    n = 200_003
    keys = rng.integers(-2**31, 2**31, 64, dtype=np.int64).astype(np.int32)
    step4 = (np.arange(64, dtype=np.int64) * 4 + 1_000_000).astype(np.int32)   # one key per slot
    flips = (keys.view(np.uint32) ^ (np.uint32(1) << rng.integers(0, 32, 64).astype(np.uint32))).view(np.int32)
    # keys made of bits 0, 8, 16 and 24 (only a multiplicative hash separates
    # them), and each with one bit flipped
    spread = np.array([(i & 1) | (i >> 1 & 1) << 8 | (i >> 2 & 1) << 16 | (i >> 3 & 1) << 24 for i in range(16)],
                      np.int32)
    sflips = (spread.view(np.uint32)[:, None] ^ (np.uint32(1) << np.arange(32, dtype=np.uint32))).view(np.int32).ravel()
    icol = np.concatenate([keys, flips, step4, step4 + 2, spread, sflips,
                           rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)])
    fvals = np.array([0.0, -0.0, np.nan, -np.nan, np.inf, -np.inf, 1.0, -1.0, 2.5, 1e-45, -1e-45, 3.4e38], np.float32)
    fbits = np.concatenate([fvals.view(np.uint32), np.array([0x7fc00001, 0xffc12345], np.uint32)])
    fcol = np.concatenate([fbits.view(np.float32), rng.standard_normal(64).astype(np.float32)])
    m = len(icol)
    icol = rng.permutation(np.resize(icol, m))
    fcol = rng.choice(fcol, m)
    t = dg.Table("slots", m, [dg.INT32, dg.FLOAT32], [icol, fcol], ["u", "u"], [None, None])
    dt = esc.device_table(t)
    preds = []
    for w in (3, 4, 5, 7, 10, 12, 20, 33, 64):
        preds.append(("in", 0, [int(v) for v in rng.choice(keys, w, replace=False)]))
    preds += [("in", 0, [int(v) for v in step4]), ("in", 0, [int(v) for v in step4[::3]]),
              ("in", 0, [0, 1, 65536]),   # no separating field, three keys: a compare list
              ("in", 0, [int(v) for v in spread]), ("in", 0, [int(v) for v in spread[::2]] + [int(keys[0])]),
              ("in", 1, [np.float32(0.0), np.float32(2.5), np.float32(np.inf)]),
              ("in", 1, [np.float32(-0.0), np.float32(1e-45), np.float32(-1.0), np.float32(np.nan)]),
              ("in", 1, [np.float32(v) for v in fvals]),
              ("in", 1, [np.float32(v) for v in rng.choice(fcol, 9)]),
              ("or", [("in", 0, [int(v) for v in keys[:6]]), ("in", 1, [np.float32(1.0), np.float32(-1.0), np.float32(0.0)])]),
              ("udf", ("add", ("col", 0), ("const", 7)), ("in", [int(v) + 7 for v in keys[10:16]]))]
    hashed = 0
    for p in preds:
        want = scan.count(t, p)
        cp = esc.Pred(dt, p)
        hashed += cp.info()["nhashed"]
        assert ctx.count(dt, cp) == want, p
        n_gpu, c, ids, outs = gpu_materialize(ctx, dt, p, [0, 1])
        wc, wids, wouts = scan.materialize(t, p, [0, 1])
        assert n_gpu == c == wc == want, p
        assert_same_rows(ids, outs, wids, wouts)
    assert hashed >= len(preds) - 2
    monkeypatch.setenv("ESC_IN_HASH_MIN", "0")
    for p in preds:
        cp = esc.Pred(dt, p)
        assert cp.info()["nhashed"] == 0
        assert ctx.count(dt, cp) == scan.count(t, p), p


def test_in_bitmaps(ctx, monkeypatch):
    """Int IN-lists that no slot field separates but that span less than
    2048 are bitmap lookups: exact at the bitmap's edges (d = 0, 2047, 2048
    and wrap-around below the smallest key), on udf values, and equal to the
    compare-list form."""
    rng = np.random.default_rng(77)
    n = 300_007
    base = 4096   # keys base + {0, 2, 66, 130}: no 6-bit field separates them
    vals = np.concatenate([np.arange(base - 40, base + 2100, dtype=np.int64),
                           [-2**31, 2**31 - 1, base - 1, base + 2047, base + 2048, base + 4096]])
    col = rng.choice(vals, n).astype(np.int32)
    other = rng.integers(-5, 5, n).astype(np.int32)
    t = dg.Table("bitmaps", n, [dg.INT32, dg.INT32], [col, other], ["u", "u"], [None, None])
    dt = esc.device_table(t)
    preds = [("in", 0, [base, base + 2, base + 66, base + 130]),
             ("in", 0, [base, base + 2, base + 66, base + 130, base + 2047]),
             ("in", 0, [base, base + 2, base + 66, base + 130, base + 2048]),    # too wide: compare list
             ("in", 0, [int(v) for v in base + np.unique(rng.integers(0, 2048, 200))[:64]]),
             ("in", 0, [-2**31, -2**31 + 2, -2**31 + 66, -2**31 + 130]),
             ("in", 0, [2**31 - 131, 2**31 - 129, 2**31 - 65, 2**31 - 1]),
             ("and", [("in", 0, [base + 1, base + 3, base + 67, base + 131]), ("gt", 1, -2)]),
             ("udf", ("add", ("col", 0), ("col", 1)), ("in", [base, base + 2, base + 66, base + 130])),
             ("or", [("in", 0, [base + 5, base + 7, base + 71, base + 135]), ("in", 0, [0, 2, 66, 130])])]
    tables = 0
    for p in preds:
        want = scan.count(t, p)
        cp = esc.Pred(dt, p)
        tables += cp.info()["nhashed"]
        assert ctx.count(dt, cp) == want, p
        n_gpu, c, ids, outs = gpu_materialize(ctx, dt, p, [0])
        wc, wids, wouts = scan.materialize(t, p, [0])
        assert n_gpu == c == wc == want, p
        assert_same_rows(ids, outs, wids, wouts)
    assert tables >= len(preds) - 1
    monkeypatch.setenv("ESC_IN_HASH_MIN", "0")
    for p in preds:
        cp = esc.Pred(dt, p)
        assert cp.info()["nhashed"] == 0
        assert ctx.count(dt, cp) == scan.count(t, p), p


def _cold_materialize(ctx, dt, p, proj, cap):
    """A materialization on a fresh workspace (no count before it)."""
    import torch
    ws = torch.zeros(ctx.workspace(dt, True, key="cold-size").numel(), dtype=torch.uint8, device="cuda")
    ids = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    outs = [torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda").view(dt.cols[j].dtype) for j in proj]
    c = ctx.materialize(dt, p, proj, ids, outs, cap, ws=ws, allow_overflow=True)
    k = min(c, cap)
    return c, ids.cpu().numpy(), [o.cpu().numpy() for o in outs], k


@pytest.mark.parametrize("n", [1, 1023, 1024, 1025, 65_537, 1_000_003])
def test_cold_materialize_single_pass_matches_three_pass(ctx, n, monkeypatch):
    """A materialization with no count before it, by the single-pass
    compaction (ESC_COLD_COMPACT=1: look-back over the tiles' published
    counts) and by the count, scan and write passes (ESC_COLD_COMPACT=0, the
    default): both and the oracle give the same count, row ids and projected values, every output
    element past the count untouched, also when the capacity cuts the output
    short.  Projections mix predicate columns (taken from registers) and
    others (read from memory)."""
    monkeypatch.setenv("ESC_COLD_COMPACT", "1")
    ctx1 = esc.Context(0)
    monkeypatch.setenv("ESC_COLD_COMPACT", "0")
    ctx3 = esc.Context(0)
    rng = np.random.default_rng(700 + n)
    cols = [np.arange(n, dtype=np.int32), rng.integers(0, 50, n).astype(np.int32),
            rng.standard_normal(n).astype(np.float32), rng.integers(-3, 4, n).astype(np.int32)]
    t = dg.Table("cold", n, [dg.INT32, dg.INT32, dg.FLOAT32, dg.INT32], cols, ["u"] * 4, [None] * 4)
    dt = esc.device_table(t)
    specs = [("lt", 1, 25), ("and", [("gt", 2, 0.5), ("in", 3, [-2, 1, 3])]), ("eq", 1, 7),
             ("or", [("between", 0, n // 3, n // 2), ("lt", 2, -1.5)]), ("lt", 0, -1), ("gt", 0, -1)]
    for i, spec in enumerate(specs):
        p = esc.Pred(dt, spec)
        proj = [2, 0, 3] if i % 2 else [1, 3]
        wc, wids, wouts = scan.materialize(t, spec, proj)
        for cap in (wc, max(wc // 3, 1)):
            c1, ids1, outs1, k1 = _cold_materialize(ctx1, dt, p, proj, cap)
            c3, ids3, outs3, k3 = _cold_materialize(ctx3, dt, p, proj, cap)
            assert c1 == c3 == wc, (spec, cap)
            assert np.array_equal(ids1, ids3) and np.array_equal(ids1[:k1], wids[:k1]), (spec, cap)
            assert (ids1[k1:] == -7).all()
            for a, b, w in zip(outs1, outs3, wouts):
                assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
                assert np.array_equal(a[:k1].view(np.uint32), w[:k1].view(np.uint32))


def test_cold_materialize_star_all_predicates(ctx, monkeypatch):
    """The 32 star predicates on 3M rows materialized cold by the single-pass
    compaction, against the oracle."""
    monkeypatch.setenv("ESC_COLD_COMPACT", "1")
    ctx = esc.Context(0)
    t = dg.table_star(3_000_000, seed=81)
    dt = esc.device_table(t)
    for i, spec in enumerate(dg.preds_star(t, 32, seed=82)):
        p = esc.Pred(dt, spec)
        wc, wids, wouts = scan.materialize(t, spec, dg.STAR_PROJECTION)
        c, ids, outs, k = _cold_materialize(ctx, dt, p, dg.STAR_PROJECTION, max(wc, 1))
        assert c == wc, i
        assert_same_rows(ids[:c], [o[:c] for o in outs], wids, wouts)


def test_simplified_programs_match_oracle(ctx, monkeypatch):
    """Predicates whose conjuncts repeat columns (the compiler intersects
    them, proves some empty and drops OR leaves that cannot hold): counts,
    row ids and projections of the simplified programs equal the oracle's,
    which evaluates the predicates as written, and equal the counts of the
    programs compiled without simplification."""
    import torch
    t = dg.table_mixed(300_007, 6, seed=97, kinds=["perm", "uniform", "zipf", "correlated", "uniform6", "lognormal"])
    dt = esc.device_table(t)
    f = np.float32
    specs = dg.preds_mixed(t, 120, seed=98, min_conj=3, max_conj=8)
    specs += [
        ("and", [("lt", 5, f(0.0)), ("gt", 5, f(-0.0))]),
        ("and", [("between", 5, f(-0.0), f(1e30)), ("lt", 5, f(3000.0)), ("gt", 5, f(100.0))]),
        ("and", [("in", 5, [f(0.0), f(2980.957), f(-1.0)]), ("gt", 5, f(-0.5))]),
        ("and", [("gt", 1, 500), ("or", [("lt", 1, 100), ("eq", 2, 7)])]),
        ("and", [("between", 1, 10, 20), ("or", [("lt", 1, 50), ("eq", 2, 7)])]),
        ("and", [("in", 1, [3, 17, 250, 9000]), ("between", 1, 10, 300), ("gt", 3, 20)]),
        ("and", [("in", 2, [1, 2, 3, 4]), ("in", 2, [3, 4, 5]), ("lt", 2, 4)]),
        ("and", [("gt", 0, 2**31 - 2), ("lt", 0, -2**31 + 1)]),
        ("and", [("gt", 4, 10), ("or", [("lt", 4, 5), ("lt", 4, 3)])]),
    ]
    simplified = [esc.Pred(dt, s_) for s_ in specs]
    monkeypatch.setenv("ESC_SIMPLIFY", "0")
    plain = [esc.Pred(dt, s_) for s_ in specs]
    monkeypatch.delenv("ESC_SIMPLIFY")
    assert sum(p.info()["constant"] == -1 for p in simplified) > sum(p.info()["constant"] == -1 for p in plain)
    assert sum(p.info()["ninsns"] for p in simplified) < sum(p.info()["ninsns"] for p in plain)
    ws = ctx.workspace(dt, True, key="simplify")
    for i, (s_, ps, pp) in enumerate(zip(specs, simplified, plain)):
        want = scan.count(t, s_)
        assert ctx.count(dt, ps, ws=ws) == want, (i, s_)
        assert ctx.count(dt, pp, ws=ws) == want, (i, s_)
        if i % 4 == 0 or i >= 120:
            cap = max(want, 1)
            ids = torch.full((cap,), -1, dtype=torch.int32, device="cuda")
            outs = [torch.zeros(cap, dtype=dt.cols[j].dtype, device="cuda") for j in (0, 5)]
            assert ctx.materialize(dt, ps, (0, 5), ids, outs, cap, ws=ws) == want
            _, wids, wouts = scan.materialize(t, s_, (0, 5))
            assert_same_rows(ids[:want].cpu().numpy(), [o[:want].cpu().numpy() for o in outs], wids, wouts)
    b = esc.Batch(ctx, [dt], simplified, [0] * len(simplified))
    assert b.count().tolist() == [scan.count(t, s_) for s_ in specs]
