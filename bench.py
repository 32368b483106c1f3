#!/usr/bin/env python3
"""Benchmark of the exact-selectivity-computation hot path on one MI355X.

Workload (one step): the 60M-row x 8-column star-schema fact table with 32
random selections of 2..5 conjuncts (date ranges, BETWEEN, IN-lists, float
comparisons); for each selection, the COUNT(*) sub-query (its result on the
host) and then its materialization with the projection (fk1, fk2, price),
enqueued without waiting.  Columns are resident
in HBM before timing starts.

value = algorithmic bytes of one step / step time, in GB/s:
  count:        k_p * N * 4        (the k_p columns predicate p reads)
  materialize:  c_p * 16 + c_p * 12
                (row ids + 3 projected values written; the 3 projected values
                of each qualifying row read).  The predicate is not evaluated
                again: the count left its truth values in the workspace.

Prints one JSON line.
"""
import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pred_columns(spec):
    cols = set()

    def walk(p):
        if p[0] in ("and", "or"):
            for q in p[1]:
                walk(q)
        elif p[0] == "udf":
            def ex(e):
                if e[0] == "col":
                    cols.add(e[1])
                elif e[0] != "const":
                    ex(e[1]); ex(e[2])
            ex(p[1])
        else:
            cols.add(p[1])
    walk(spec)
    return cols


def profile_record(name):
    """key: value lines of a counter record under profiles/, or None when the
    kernel sources it names changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.split("#")[0].strip()
    h = hashlib.sha256()
    for src in kv.get("kernel_sources", "").split():
        fp = os.path.join(ROOT, src)
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if h.hexdigest() != kv.get("kernel_sources_sha256"):
        return None
    return kv


def counter_traffic():
    """HBM bytes per count-kernel launch measured with the FETCH_SIZE and
    WRITE_SIZE counters (profiles/count_kernel_star60M_pmc.txt), or None when
    the kernel sources changed since the counters were taken."""
    kv = profile_record("count_kernel_star60M_pmc.txt")
    return int(kv["traffic_bytes_per_launch"]) if kv else None


_ORACLE_TABLE = None


def _oracle_init(meta):
    global _ORACLE_TABLE
    from paper_1901_01488_amd import datagen as dg
    name, nrows, dtypes, paths, kinds, domain = meta
    cols = [np.load(p, mmap_mode="r") for p in paths]
    _ORACLE_TABLE = dg.Table(name, nrows, dtypes, cols, kinds, domain)


def _oracle_one(job):
    from oracle import scan
    i, spec = job
    return i, scan.count(_ORACLE_TABLE, spec)


def oracle_counts(host, specs, idx, what):
    """Oracle counts of specs[i] for i in idx: one single-threaded oracle per
    worker process.  The workers are fresh interpreters (no GPU state) that
    map the host table's columns from files written once."""
    import multiprocessing as mp
    import shutil
    import tempfile
    d = tempfile.mkdtemp(prefix="esc_oracle_")
    try:
        paths = []
        for j, c in enumerate(host.cols):
            pth = os.path.join(d, f"c{j}.npy")
            np.save(pth, np.ascontiguousarray(c))
            paths.append(pth)
        meta = (host.name, host.nrows, list(host.dtypes), paths, list(host.kinds), list(host.domain))
        workers = max(1, min(16, os.cpu_count() or 1, len(idx)))
        out = {}
        t0 = time.perf_counter()
        with mp.get_context("spawn").Pool(workers, initializer=_oracle_init, initargs=(meta,)) as pool:
            jobs = [(int(i), specs[i]) for i in idx]
            for j, (i, c) in enumerate(pool.imap_unordered(_oracle_one, jobs, chunksize=1)):
                out[i] = c
                if (j + 1) % max(1, len(idx) // 10) == 0:
                    log(f"{what}: oracle {j + 1}/{len(idx)}")
        return out, workers, time.perf_counter() - t0
    finally:
        shutil.rmtree(d, ignore_errors=True)


def cpu_baseline_parallel(t_host, preds, counts):
    """The oracle on P cores: the 32 predicates over all rows, one
    single-threaded oracle per worker process (P = the host's cores, at most
    16), scaled to GB/s of algorithmic bytes; its counts are checked against
    the library's."""
    idx = list(range(len(preds)))
    got, workers, sec = oracle_counts(t_host, preds, idx, "multicore baseline")
    nbytes = sum(len(pred_columns(p)) * t_host.nrows * 4 for p in preds)
    return {"value": round(nbytes / sec / 1e9, 3), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": f"count(*) of all {len(preds)} predicates over all {t_host.nrows} rows, one process per "
                      f"core ({workers}), {sec:.1f} s including worker start",
            "count_errors": int(sum(int(counts[i]) != got[i] for i in idx))}


def cpu_baseline(t_host, preds, budget_s=25.0):
    """The oracle (single thread) on the first rows of the same table, all 32
    predicates, count only; scaled to GB/s of algorithmic bytes."""
    from oracle import scan
    from paper_1901_01488_amd import datagen as dg
    n = t_host.nrows
    sub = dg.Table("sample", n, t_host.dtypes, [c[:n] for c in t_host.cols]).host()
    t0 = time.perf_counter()
    nbytes = 0
    done = 0
    for p in preds:
        scan.count(sub, p)
        nbytes += len(pred_columns(p)) * n * 4
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"count(*) of {done} of the 32 predicates over the first {n} rows, one thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--rows", type=int, default=60_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the bounded learned-gate and planning extras")
    ap.add_argument("--learned", action="store_true", help="learned-gate workload (100M x 6, 200K labels)")
    ap.add_argument("--planning", action="store_true", help="planning workload (1,000 three-table queries)")
    ap.add_argument("--copy-ref", action="store_true", help="1 GiB device copy (counter calibration)")
    ap.add_argument("--batched", action="store_true", help="batched workload only (256 sub-queries, 8 tables)")
    ap.add_argument("--policy", action="store_true", help="materialization policy: calibrated cost model vs measured costs")
    ap.add_argument("--join", action="store_true", help="star join over ESC temporary tables (10M / 100M build, 1B probe)")
    ap.add_argument("--sweeps", action="store_true", help="selectivity sweep (2*10^8-row permutation) and "
                                                               "1..5-attribute sweep (star table)")
    ap.add_argument("--typed", action="store_true", help="TEXT / DECIMAL(15,2) predicates (60M rows, 64 predicates)")
    ap.add_argument("--mlp", action="store_true", help="MLP kernels alone: inference per 4,096 batch, training steps")
    ap.add_argument("--train-preds", type=int, default=200_000)
    ap.add_argument("--queries", type=int, default=1000)
    args = ap.parse_args()
    if args.copy_ref:
        return copy_reference()
    if args.batched:
        return batched_workload()
    if args.mlp:
        return mlp_workload()
    if args.learned:
        return learned_workload(args)
    if args.planning:
        return planning_workload(args)
    if args.policy:
        return policy_workload()
    if args.join:
        return join_workload()
    if args.typed:
        return typed_workload()
    if args.sweeps:
        return sweeps_workload()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only (sharding by rows across GPUs is designed, "
                                   "not implemented): --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc

    torch.cuda.init()
    dev = "cuda:0"
    log("generating the star table on the device")
    t = dg.table_star(args.rows, device=dev)
    preds = dg.preds_star(t, 32)
    dt = esc.Table(t.nrows, t.dtypes, t.cols)
    torch.cuda.synchronize()
    ctx = esc.Context(0)
    stream = torch.cuda.current_stream()
    cps = [esc.Pred(dt, p) for p in preds]
    proj = dg.STAR_PROJECTION
    ks = [len(pred_columns(p)) for p in preds]

    # capacities from one exact count each (outside timing)
    counts = [ctx.count(dt, p) for p in cps]
    cap = max(max(counts), 1)
    rowids = torch.empty(cap, dtype=torch.int32, device=dev)
    outs = [torch.empty(cap, dtype=dt.cols[j].dtype, device=dev) for j in proj]
    ws = ctx.workspace(dt, True)
    ws2 = [ws, ctx.workspace(dt, True, key="step-1")]

    dmat = torch.zeros(len(cps), dtype=torch.int64, device=dev)

    def step():
        # each count comes back to the host (the push-down decision needs
        # it) and its materialization is enqueued behind it without a wait;
        # the next selection's count is enqueued before the host waits, so
        # the GPU does not idle while the host decides (two workspaces in
        # turn keep each count's tiles for its own materialization)
        ctx.count_begin(dt, cps[0], ws2[0], 0, stream=stream)
        for i, p in enumerate(cps):
            if i + 1 < len(cps):
                ctx.count_begin(dt, cps[i + 1], ws2[(i + 1) % 2], (i + 1) % 2, stream=stream)
            ctx.count_end(i % 2)
            ctx.materialize_async(dt, p, proj, rowids, outs, cap, dmat[i:i + 1], ws2[i % 2], stream=stream)

    N = t.nrows
    step_bytes = 0
    for k, c in zip(ks, counts):
        step_bytes += k * N * 4                                  # count
        step_bytes += c * 4 * (1 + len(proj)) + c * 4 * len(proj)   # materialize

    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("timed steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / args.steps * 1e3
    value = step_bytes / (el / args.steps) / 1e9
    assert dmat.cpu().tolist() == counts

    # a cold materialization of every predicate (no count before it): the
    # single-pass compaction against count + scan + write, event-timed
    # back to back on the stream
    log("cold materialization")
    cold = {}
    os.environ["ESC_COLD_COMPACT"] = "1"
    ctx1 = esc.Context(0)
    del os.environ["ESC_COLD_COMPACT"]
    wsc = torch.zeros(ws.numel(), dtype=torch.uint8, device=dev)
    for name, cx in (("single_pass", ctx1), ("three_pass", ctx)):
        times = []
        for rep in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            esc.check(esc.lib().esc_workspace_init(cx.h, esc.ctypes.c_void_p(wsc.data_ptr()), wsc.numel(), None))
            e0.record(stream)
            for i, p in enumerate(cps):
                # every call is cold: the previous predicate's tiles are not this one's
                cx.materialize_async(dt, p, proj, rowids, outs, cap, dmat[i:i + 1], wsc, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
            assert dmat.cpu().tolist() == counts
        cold[f"cold_materialize_32_{name}_ms"] = round(float(np.median(times)), 3)
    del ctx1, wsc

    # dominant kernel: the count scan, timed with HIP events on the stream it
    # runs on.  The 32 predicates' launches run back to back between two
    # events after a 1 GiB read (a reduction over an unrelated buffer) has
    # evicted the 256 MB last-level cache without leaving dirty lines; the
    # table (1.9 GB) is far larger than that cache and every launch scans it
    # from the start, so each launch reads its columns from HBM (the counters
    # confirm it).  Median of 3 repetitions.  Also reported: every launch
    # timed alone after its own eviction (includes per-launch event latency).
    log("count-kernel timing")
    dcount = torch.zeros(len(cps), dtype=torch.int64, device=dev)
    scratch = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # a float32 sum reads it with no int64 copy
    cws = ctx.workspace(dt, False, key="count")
    kern_bytes = [k * N * 4 for k in ks]
    reps = []
    for _ in range(3):
        scratch.sum()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i, p in enumerate(cps):
            ctx.count_async(dt, p, dcount[i:i + 1], cws, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        reps.append(e0.elapsed_time(e1))
        assert dcount.cpu().tolist() == counts
    b2b_ms = float(np.median(reps))
    achieved = sum(kern_bytes) / (b2b_ms / 1e3) / 1e9
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cps]
    for i, p in enumerate(cps):
        scratch.sum()
        torch.cuda.synchronize()
        ev[i][0].record(stream)
        ctx.count_async(dt, p, dcount[i:i + 1], cws, stream=stream)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    single_ms = [a.elapsed_time(b) for a, b in ev]
    assert dcount.cpu().tolist() == counts
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counter_traffic(),
                "kernel": "count_kernel (all instantiations)",
                "avg_launch_us": round(b2b_ms / len(cps) * 1e3, 2),
                "bytes_per_launch": int(sum(kern_bytes) / len(kern_bytes)),
                "single_launch_cold_GBps": round(sum(kern_bytes) / (sum(single_ms) / 1e3) / 1e9, 1)}
    del scratch

    extras = dict(cold)
    if not args.no_extras:
        for name, fn in (("conjuncts", lambda: conjunct_split(ctx, dt, cps, kern_bytes)),
                         ("plain_latency", lambda: plain_latency(ctx, esc, dg, torch, dev)),
                         ("batched", lambda: batched_vs_plain(ctx, esc, dg, torch, dev))):
            try:
                extras.update(fn())
            except Exception as e:   # an extra must not hide the headline line; the error is reported
                extras[name + "_error"] = repr(e)[:300]
            torch.cuda.empty_cache()

    if not args.no_extras and not args.no_learned:
        # the learned gate and the planning load, bounded (the full runs are
        # --learned and --planning): full-size estimator, fewer oracle checks;
        # planning estimators trained on fewer labels, capacity runs only
        for name, fn in (("learned", lambda: learned_leg(ctx, 200_000, oracle_random=100, oracle_routed=100)),
                         ("planning", lambda: planning_leg(ctx, 1000, train_n=(20_000, 20_000, 4_000), epochs=20,
                                                           offered=False, oracle_rs=32, oracle_p=0)),
                         ("planning_nonempty", lambda: planning_leg(ctx, 1000, train_n=(20_000, 20_000, 4_000),
                                                                    epochs=20, offered=False, oracle_rs=32,
                                                                    oracle_p=0, gen="anchored"))):
            try:
                log(f"extra: {name}")
                extras[name] = fn()
            except Exception as e:
                extras[name + "_error"] = repr(e)[:300]
            torch.cuda.empty_cache()

    line = {
        "metric": "ESC scan GB/s vs HBM peak; predicates/s batched vs plain; p50/p99 ms/query",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/float32 compares, u64 counts", "data": "synthetic (seeded; star-schema stand-in)",
        "config": {"workload": "star fact table 60M x 8 cols, 32 predicates, count + materialize each",
                   "rows": N, "predicates": len(preds), "parallelism": "1 GPU"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline")
        host = t.host()
        line["cpu_baseline"] = cpu_baseline(host, preds)
        log("cpu baseline, one process per core")
        line["cpu_baseline_multicore"] = cpu_baseline_parallel(host, preds, counts)
    line["extras"] = extras
    print(json.dumps(line), flush=True)


def conjunct_split(ctx, dt, cps, kern_bytes, reps=3):
    """Per-conjunct and prefix counts of the 32 star predicates (one scan
    each): wall time of the blocking call against the plain count's."""
    for p in cps:
        ctx.count_conjuncts(dt, p)
    tc, tp = [], []
    for _ in range(reps):
        a = time.perf_counter()
        for p in cps:
            ctx.count_conjuncts(dt, p)
        tc.append(time.perf_counter() - a)
        a = time.perf_counter()
        for p in cps:
            ctx.count(dt, p)
        tp.append(time.perf_counter() - a)
    c, q = float(np.median(tc)), float(np.median(tp))
    return {"split_conjuncts_GBps": round(sum(kern_bytes) / c / 1e9, 1),
            "split_conjuncts_ms_per_predicate": round(c / len(cps) * 1e3, 3),
            "plain_count_ms_per_predicate": round(q / len(cps) * 1e3, 3)}


def batched_vs_plain(ctx, esc, dg, torch, dev, reps=20):
    """256 selectivity sub-queries over 8 tables of 10K..200M rows: one
    autotuned graph launch of the batched kernel vs 256 plain count calls
    (each synchronous, and all queued then one synchronisation)."""
    log("batched workload: generating tables")
    tabs = dg.tables_batched(device=dev)
    preds, owner = dg.preds_batched(tabs)
    dts = [esc.Table(t.nrows, t.dtypes, t.cols) for t in tabs]
    cps = [esc.Pred(dts[o], p) for p, o in zip(preds, owner)]
    torch.cuda.synchronize()
    log("batched workload: autotune")
    t0 = time.perf_counter()
    b = esc.Batch(ctx, dts, cps, owner, autotune=True)
    tune_s = time.perf_counter() - t0
    got = b.count()
    ws = [ctx.workspace(d, False, key=("bt", i)) for i, d in enumerate(dts)]
    plain = [ctx.count(dts[o], p, ws=ws[o]) for p, o in zip(cps, owner)]
    assert got.tolist() == plain
    tb = []
    for _ in range(reps):
        a = time.perf_counter()
        b.count()
        tb.append(time.perf_counter() - a)
    ts = []
    for _ in range(3):
        a = time.perf_counter()
        for p, o in zip(cps, owner):
            ctx.count(dts[o], p, ws=ws[o])
        ts.append(time.perf_counter() - a)
    dout = torch.zeros(len(cps), dtype=torch.int64, device=dev)
    aws = ctx.workspace(dts[0], False, key="ba")   # one stream: launches run in order
    ta = []
    for _ in range(3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i, (p, o) in enumerate(zip(cps, owner)):
            ctx.count_async(dts[o], p, dout[i:i + 1], aws)
        torch.cuda.synchronize()
        ta.append(time.perf_counter() - a)
    assert dout.cpu().tolist() == plain
    n = len(cps)
    tbm, tsm, tam = float(np.median(tb)), float(np.median(ts)), float(np.median(ta))
    decided = [p.info()["constant"] != 0 for p in cps]
    scanned_rows = sum(tabs[o].nrows for o, d in zip(owner, decided) if not d)
    # the same predicates compiled as written (no intersection of conjuncts
    # on one column): every one is scanned
    log("batched workload: without conjunct simplification")
    os.environ["ESC_SIMPLIFY"] = "0"
    try:
        raw = [esc.Pred(dts[o], p) for p, o in zip(preds, owner)]
    finally:
        del os.environ["ESC_SIMPLIFY"]
    o_ = b.opts()
    braw = esc.Batch(ctx, dts, raw, owner, rows_per_thread=o_["rows_per_thread"], group=o_["group"],
                     chunk_rows=o_["chunk_rows"], max_cols=o_["max_cols"])
    assert braw.count().tolist() == plain
    tr = []
    for _ in range(reps):
        a = time.perf_counter()
        braw.count()
        tr.append(time.perf_counter() - a)
    tra = []
    for _ in range(3):
        torch.cuda.synchronize()
        a = time.perf_counter()
        for i, (p, o) in enumerate(zip(raw, owner)):
            ctx.count_async(dts[o], p, dout[i:i + 1], aws)
        torch.cuda.synchronize()
        tra.append(time.perf_counter() - a)
    assert dout.cpu().tolist() == plain
    trm, tram = float(np.median(tr)), float(np.median(tra))
    bytes_batched = 0
    for ti, t in enumerate(tabs):
        used = set()
        for p, o in zip(preds, owner):
            if o == ti:
                used |= pred_columns(p)
        bytes_batched += len(used) * t.nrows * 4
    return {"batched_256_predicates_per_s": round(n / tbm, 1),
            "plain_sync_predicates_per_s": round(n / tsm, 1),
            "plain_async_predicates_per_s": round(n / tam, 1),
            "batched_speedup_vs_best_plain": round(min(tsm, tam) / tbm, 2),
            "batched_ms": round(tbm * 1e3, 3), "batched_GBps_distinct_columns": round(bytes_batched / tbm / 1e9, 1),
            "batched_opts": b.opts(), "autotune_s": round(tune_s, 2),
            "batched_decided_by_the_compiler": int(sum(decided)),
            "batched_scanned_row_predicates": int(scanned_rows),
            "batched_row_predicates_per_s": round(scanned_rows / tbm, 1),
            "without_simplification": {"batched_ms": round(trm * 1e3, 3),
                                       "batched_predicates_per_s": round(n / trm, 1),
                                       "plain_async_predicates_per_s": round(n / tram, 1),
                                       "batched_speedup_vs_plain_async": round(tram / trm, 2),
                                       "batched_row_predicates_per_s": round(32 * sum(t.nrows for t in tabs) / trm, 1)},
            # from the SQ counters of profiles/batch_kernel_256preds_8tables.txt (None once the kernel changed)
            "batched_valu_issue_fraction": (lambda kv: float(kv["valu_issue_fraction (SQ_INSTS_VALU x 4 / (1024 x "
                                                            "cycles))"]) if kv else None)(
                profile_record("batch_kernel_256preds_8tables.txt"))}


def cpu_baseline_plain(t, want):
    """cpu_baseline leg of the plain-latency extra: the oracle's count of the
    Section 1 selection on the same 1M-row table, one host thread."""
    from oracle import scan
    from paper_1901_01488_amd import datagen as dg
    a = time.perf_counter()
    got = scan.count(t, dg.pred_plain(t, 0))
    oracle_s = time.perf_counter() - a
    assert got == want
    return {"value": round(oracle_s / t.nrows * 1e9, 2), "unit": "ns/row", "cores": 1, "kind": "oracle",
            "sample": "count(*) of the Section 1 selection over all 1M rows"}


def plain_latency(ctx, esc, dg, torch, dev, reps=1000):
    """The Section 1 selection on a 1M-row table: wall latency of esc_count
    and esc_materialize (launch to result on the host), p50/p99."""
    t = dg.table_plain(1_000_000)
    dt = esc.device_table(t, dev)
    p = esc.Pred(dt, dg.pred_plain(t, 0))
    n = ctx.count(dt, p)
    ids = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    outs = [torch.empty(max(n, 1), dtype=torch.int32, device=dev) for _ in dg.PLAIN_PROJECTION]
    ws = ctx.workspace(dt, True, key="plain")
    # the caller holds its stream, as a serving loop would (looking up
    # torch's current stream costs microseconds of Python per call)
    st = torch.cuda.current_stream()
    for _ in range(20):
        ctx.count(dt, p, ws=ws, stream=st)
        ctx.materialize(dt, p, dg.PLAIN_PROJECTION, ids, outs, n, ws=ws, stream=st)
    tc, tm = [], []
    for _ in range(reps):
        a = time.perf_counter()
        ctx.count(dt, p, ws=ws, stream=st)
        b = time.perf_counter()
        ctx.materialize(dt, p, dg.PLAIN_PROJECTION, ids, outs, n, ws=ws, stream=st)
        c = time.perf_counter()
        tc.append((b - a) * 1e6)
        tm.append((c - b) * 1e6)
    # a materialization with no count before it: single pass (look-back
    # compaction, a context made with ESC_COLD_COMPACT=1) against count +
    # scan + write (the default; its workspace's tile record is dropped
    # before each call, outside the timing)
    cold = {}
    os.environ["ESC_COLD_COMPACT"] = "1"
    ctx1 = esc.Context(0)
    del os.environ["ESC_COLD_COMPACT"]
    for name, cx in (("single_pass", ctx1), ("three_pass", ctx)):
        wsc = torch.zeros(ws.numel(), dtype=torch.uint8, device=dev)
        tt = []
        for i in range(reps // 2 + 20):
            if name == "three_pass":
                esc.check(esc.lib().esc_workspace_init(cx.h, esc.ctypes.c_void_p(wsc.data_ptr()), wsc.numel(), None))
                torch.cuda.synchronize()
            a = time.perf_counter()
            got = cx.materialize(dt, p, dg.PLAIN_PROJECTION, ids, outs, n, ws=wsc)
            tt.append((time.perf_counter() - a) * 1e6)
            assert got == n
        tt = tt[20:]
        cold[f"plain_1M_cold_materialize_{name}_us_p50"] = round(float(np.percentile(tt, 50)), 1)
        cold[f"plain_1M_cold_materialize_{name}_us_p99"] = round(float(np.percentile(tt, 99)), 1)
    return {"plain_1M_cpu_baseline": cpu_baseline_plain(t, n), **cold,
            "plain_1M_count_us_p50": round(float(np.percentile(tc, 50)), 1),
            "plain_1M_count_us_p99": round(float(np.percentile(tc, 99)), 1),
            "plain_1M_materialize_us_p50": round(float(np.percentile(tm, 50)), 1),
            "plain_1M_materialize_us_p99": round(float(np.percentile(tm, 99)), 1)}



def batched_workload():
    """The batched workload alone: one JSON line."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc
    torch.cuda.init()
    ctx = esc.Context(0)
    r = batched_vs_plain(ctx, esc, dg, torch, "cuda:0")
    r["workload"] = "batched: 256 sub-queries over 8 tables of 10K..200M rows (376M rows), count only"
    print(json.dumps(r), flush=True)


def copy_reference():
    """A plain 1 GiB device-to-device copy, for calibrating HBM byte counters."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4, "launches": 3}))


def mlp_workload():
    """The estimator's kernels alone on seeded synthetic features: inference
    of a 4,096-row batch (one launch) and training steps of 256 and 1,024
    rows (two kernels and a step advance per step, replayed from a graph),
    event-timed; TFLOP/s against the bf16 dense MFMA peak."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc
    torch.cuda.init()
    ctx = esc.Context(0)
    m = esc.MLP(ctx, dg.mlp_init(dg.MLP_SEED))
    g = torch.Generator(device="cuda:0").manual_seed(3)
    x = torch.randn(4096, 64, device="cuda:0", generator=g)
    out = torch.empty(4096, device="cuda:0")
    for _ in range(20):
        m.predict(x, out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(200):
        m.predict(x, out)
    e1.record()
    torch.cuda.synchronize()
    infer_us = e0.elapsed_time(e1) / 200 * 1e3
    fwd_flop = 2 * (64 * 256 + 2 * 256 * 256 + 256)
    res = {"workload": "MLP 64-256-256-256-1, bf16 MFMA / fp32 accumulate",
           "inference_us_per_4096": round(infer_us, 2),
           "inference_tflops": round(4096 * fwd_flop / (infer_us * 1e-6) / 1e12, 1),
           "peak_tflops_bf16_dense": 2500.0}
    n = 200_000
    X = torch.randn(n, 64, device="cuda:0", generator=g)
    Y = torch.randn(n, device="cuda:0", generator=g)
    for batch in (256, 1024):
        order = torch.from_numpy(dg.minibatch_order(n, batch, 2, seed=3)).cuda()
        steps = len(order) // batch
        m.train(X, Y, order, 10, batch, want_loss=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.train(X, Y, order, steps, batch, want_loss=False)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / steps * 1e6
        # forward + backward (two input-gradient and three weight-gradient products)
        flop = batch * (3 * fwd_flop - 2 * 64 * 256)
        res[f"train_us_per_step_batch{batch}"] = round(us, 1)
        res[f"train_tflops_batch{batch}"] = round(flop / (us * 1e-6) / 1e12, 2)
    print(json.dumps(res), flush=True)


def learned_workload(args):
    """Learned gate at full size: labels, training, q-error and the oracle's
    check of 1,000 random labels and every routed test predicate."""
    import torch
    torch.cuda.init()
    from paper_1901_01488_amd import esc
    ctx = esc.Context(0)
    r = learned_leg(ctx, args.train_preds, oracle_random=1000, oracle_routed=None)
    print(json.dumps(r), flush=True)


def learned_leg(ctx, ntrain, oracle_random, oracle_routed):
    """Learned gate on a 100M x 6 correlated / skewed table: exact labels by
    the batched scan, GPU training, q-error on a held-out batch of 4,096,
    routing and exact fallback.  Predicates are conjunctions built around
    sampled rows (every one selects at least one row).  Routed predicates are
    counted again by the plain count kernel (all of them) and by the oracle
    (oracle_routed of them, None = all), beside oracle_random random labels."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc, learned
    dev = "cuda:0"
    n = 100_000_000
    log("learned: table")
    t = dg.table_learned(n, device=dev)
    dt = esc.Table(t.nrows, t.dtypes, t.cols)
    catalog = learned.Catalog.of(t, seed=dg.pred_seed(3) + 1)
    nval, ntest = 8192, 4096
    log("learned: predicates")
    t0 = time.perf_counter()
    specs = dg.preds_anchored(t, ntrain + nval + ntest, seed=dg.pred_seed(3))
    cps = [esc.Pred(dt, p) for p in specs]
    gen_s = time.perf_counter() - t0
    log("learned: labels")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = learned.exact_counts(ctx, dt, cps)
    label_s = time.perf_counter() - t0
    log("learned: features + training")
    est = learned.Estimator(ctx, dt, catalog, dg.mlp_init(dg.MLP_SEED))
    t0 = time.perf_counter()
    x = est.features(cps)
    feat_s = time.perf_counter() - t0
    y = learned.labels(counts, n)
    tr, va, te = slice(0, ntrain), slice(ntrain, ntrain + nval), slice(ntrain + nval, None)
    phases = [(20, 1e-3), (10, 2e-4), (10, 4e-5)]
    loss, train_s = est.fit(x[tr], y[tr], phases, batch=256, order_seed=dg.MLP_SEED)
    steps = sum(e for e, _ in phases) * (ntrain // 256)
    beta = learned.validation_beta(est.predict(x[va]), counts[va], n)
    xt = torch.from_numpy(x[te]).to(dev)
    out = torch.empty(ntest, dtype=torch.float32, device=dev)
    for _ in range(5):
        est.mlp.predict(xt, out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(20):
        est.mlp.predict(xt, out)
    ev1.record()
    torch.cuda.synchronize()
    infer_us = ev0.elapsed_time(ev1) / 20 * 1e3
    yhat = out.cpu().numpy()
    q = learned.q_error(learned.c_hat(yhat, n), counts[te], n)
    route = esc.gate_pushdown(yhat, n, 0.05, beta, 1_000_000)
    idx = np.flatnonzero(route) + te.start
    # the routed predicates' exact fallback: the batched labels against the
    # plain count kernel, one esc_count each
    ws = ctx.workspace(dt, False, key="learned-count")
    plain = np.array([ctx.count(dt, cps[i], ws=ws) for i in idx], np.uint64)
    rng = np.random.default_rng(0)
    pick = idx if oracle_routed is None or len(idx) <= oracle_routed else rng.choice(idx, oracle_routed, replace=False)
    check = sorted(set(int(i) for i in rng.choice(len(counts), oracle_random, replace=False)) |
                   set(int(i) for i in pick))
    got, workers, oracle_s = oracle_counts(t.host(), specs, check, "learned")
    oracle_errors = sum(int(counts[i]) != got[i] for i in check)
    flops = 4096 * 2 * (64 * 256 + 2 * 256 * 256 + 256)
    return {
        "workload": "learned gate: 100M x 6 table, %d training predicates, held-out batch of 4096" % ntrain,
        "label_s": round(label_s, 2), "label_row_predicates_per_s": round(len(cps) * n / label_s, 1),
        "features_us_per_predicate": round(feat_s / len(cps) * 1e6, 2),
        "train_s": round(train_s, 2), "train_steps": steps, "train_us_per_step": round(train_s / steps * 1e6, 1),
        "schedule": "batch 256; epochs@lr " + ", ".join(f"{e}@{l:g}" for e, l in phases),
        "final_loss": float(np.mean(loss[-50:])), "zero_count_fraction": float((counts == 0).mean()),
        "inference_us_per_4096": round(infer_us, 1), "inference_tflops": round(flops / (infer_us * 1e-6) / 1e12, 3),
        "qerror_median": float(np.median(q)), "qerror_p90": float(np.quantile(q, 0.9)),
        "qerror_p99": float(np.quantile(q, 0.99)), "qerror_max": float(q.max()), "beta": beta,
        "routed_fraction": float(route.mean()),
        "routed_count_errors": int((plain != counts[idx]).sum()) + sum(int(counts[i]) != got[i] for i in pick),
        "cpu_baseline": {"value": round(len(check) * n / oracle_s, 1), "unit": "row-predicates/s",
                         "cores": workers, "kind": "oracle",
                         "sample": f"{oracle_random} random labels + {len(pick)} of the {len(idx)} routed test "
                                   "predicates, one process per core",
                         "checked": len(check), "errors": oracle_errors, "seconds": round(oracle_s, 1)},
        "predicate_gen_s": round(gen_s, 1)}


def planning_workload(args):
    """Planning load at full size: offered load and capacity, both probe
    settings, the oracle on every selection of R and S and 48 on P."""
    import torch
    torch.cuda.init()
    from paper_1901_01488_amd import esc
    ctx = esc.Context(0)
    r = planning_leg(ctx, args.queries, train_n=(100_000, 100_000, 20_000), epochs=20, offered=True,
                     oracle_rs=None, oracle_p=48)
    r2 = planning_leg(ctx, args.queries, train_n=(100_000, 100_000, 20_000), epochs=20, offered=False,
                      oracle_rs=None, oracle_p=48, gen="anchored")
    print(json.dumps({"planning": r, "planning_nonempty": r2}), flush=True)


def planning_queries(dg, table, count, seed, gen):
    """Selections of one table: `mixed` = 2-6 conjuncts with random
    constants (most select nothing), `anchored` = 2-4 conjuncts on distinct
    columns built around a sampled row (every selection keeps >= 1 row)."""
    if gen == "anchored":
        return dg.preds_anchored(table, count, seed=seed, min_conj=2, max_conj=4)
    return dg.preds_mixed(table, count, seed=seed, min_conj=2, max_conj=6)


def planning_leg(ctx, nq, train_n, epochs, offered, oracle_rs, oracle_p, gen="mixed"):
    """nq arriving three-table queries (10M / 100M / 1B rows): plain
    per-selection counts vs micro-batched graph launches vs batched + gate,
    every mode on the same work.  oracle_rs: selections of R and S the oracle
    checks (None = all); oracle_p: selections of P it checks; gen: the query
    generator (planning_queries)."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc, learned, planning
    dev = "cuda:0"
    log("planning: tables")
    tabs = dg.tables_planning(device=dev)
    dts = [esc.Table(t.nrows, t.dtypes, t.cols) for t in tabs]
    qs = [planning_queries(dg, t, nq, dg.pred_seed(4) + i, gen) for i, t in enumerate(tabs)]
    queries = list(zip(*qs))
    arrivals = dg.poisson_arrivals(nq, 2000.0, seed=dg.pred_seed(4))
    ests = []
    t0 = time.perf_counter()
    for i, (t, dt) in enumerate(zip(tabs, dts)):
        log(f"planning: estimator {i}")
        specs = planning_queries(dg, t, train_n[i], dg.pred_seed(4) + 100 + i, gen)
        cps = [esc.Pred(dt, p) for p in specs]
        cnt = learned.exact_counts(ctx, dt, cps)
        e = learned.Estimator(ctx, dt, learned.Catalog.of(t, seed=11 + i), dg.mlp_init(dg.MLP_SEED))
        x = e.features(cps)
        e.train(x, learned.labels(cnt, t.nrows), epochs=epochs, batch=1024, lr=1e-3, order_seed=11 + i)
        ests.append(e)
    offline_s = time.perf_counter() - t0
    # every mode does identical work: the probe relation's selection is
    # counted by no mode (exact_probe 0: no plan depends on it) or by all (1)
    modes = {}
    kinds = [("offered", 1.0), ("capacity", 50.0)] if offered else [("capacity", 50.0)]
    for kind, speed in kinds:
        w = planning.Workload(ctx, dts, queries, arrivals / speed)
        for probe in (0, 1):
            log(f"planning: {kind}, exact_probe {probe}")
            gc = planning.GateConfig(beta=1.5, exact_probe=bool(probe))
            strict = planning.GateConfig(beta=1.5, exact_probe=bool(probe), tie_sel=0.0)
            modes[(kind, probe)] = (w.run_plain(exact_probe=bool(probe)), w.run_batched(exact_probe=bool(probe)),
                                    w.run_batched(gate=True, estimators=ests, gcfg=gc),
                                    w.run_batched(gate=True, estimators=ests, gcfg=strict))
    plain = modes[(kinds[0][0], 1)][0]   # counts of all three selections
    count_errors = 0
    for (kind, probe), (pl, ba, ga, gs) in modes.items():
        cols = [0, 1, 2] if probe else [0, 1]
        count_errors += int((pl["counts"][:, cols] != plain["counts"][:, cols]).sum())
        count_errors += int((ba["counts"][:, cols] != plain["counts"][:, cols]).sum())
        for g in (ga, gs):
            ex = g["routed"] | g["known"]
            count_errors += int((g["counts"][ex] != plain["counts"][ex]).sum())
    nrows = [t.nrows for t in tabs]
    exact_sel = plain["counts"] / np.array(nrows, np.float64)

    def agreement(gated, gcfg):
        r = gated["routed"] | gated["known"]   # counted, or decided by the compiler
        est_sel = np.where(r, gated["counts"] / np.array(nrows, np.float64), np.exp(gated["est"]))
        ex, es = planning.plans(exact_sel, nrows, gcfg), planning.plans(est_sel, nrows, gcfg)
        return (float(np.mean([planning.agree(a, b, s, gcfg) for a, b, s in zip(ex, es, exact_sel)])),
                float(np.mean([a == b for a, b in zip(ex, es)])))

    tie_cfg = planning.GateConfig(beta=1.5)
    agree_tie, agree_tie_strict = agreement(modes[(kinds[0][0], 0)][2], tie_cfg)
    agree_strict, _ = agreement(modes[(kinds[0][0], 0)][3], planning.GateConfig(beta=1.5, tie_sel=0.0))
    empty = [float(np.mean(plain["counts"][:, t] == 0)) for t in range(3)]
    decided = [float(np.mean(modes[(kinds[0][0], 0)][2]["known"][:, t])) for t in range(3)]
    ties = float(np.mean((exact_sel[:, 0] <= tie_cfg.tie_sel) & (exact_sel[:, 1] <= tie_cfg.tie_sel)))
    # the oracle checks exact counts of R and S (all, or a seeded sample) and
    # a seeded sample of P
    oracle_errors, oracle_checked, oracle_rows, oracle_s, workers = 0, 0, 0, 0.0, 1
    rng = np.random.default_rng(5)
    for ti, tab in enumerate(tabs):
        want = oracle_p if ti == 2 else oracle_rs
        if want == 0:
            continue
        idx = list(range(nq)) if want is None else sorted(rng.choice(nq, min(want, nq), replace=False).tolist())
        log(f"planning: oracle on table {ti} ({len(idx)} selections)")
        got, workers, sec = oracle_counts(tab.host(), [q[ti] for q in queries], idx, f"planning table {ti}")
        oracle_errors += sum(int(plain["counts"][i, ti]) != got[i] for i in idx)
        oracle_checked += len(idx)
        oracle_rows += len(idx) * tab.nrows
        oracle_s += sec
    strip = lambda d: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in d.items()
                       if k not in ("counts", "est", "routed", "known")}
    table = {}
    for (kind, probe), (pl, ba, ga, gs) in modes.items():
        table[f"{kind}_exact_probe{probe}"] = {
            "plain": strip(pl), "batched": strip(ba), "batched_gate": strip(ga), "batched_gate_no_ties": strip(gs),
            "batched_speedup_vs_plain": round(ba["predicates_per_s"] / pl["predicates_per_s"], 2),
            "gate_speedup_vs_plain": round(ga["predicates_per_s"] / pl["predicates_per_s"], 2),
            "gate_speedup_vs_batched": round(ga["predicates_per_s"] / ba["predicates_per_s"], 2),
            "gate_no_ties_speedup_vs_plain": round(gs["predicates_per_s"] / pl["predicates_per_s"], 2)}
    return {
        "workload": f"planning: {nq} three-table queries over 10M / 100M / 1B rows, Poisson arrivals 2000/s; "
                    f"selections: {'2-4 conjuncts around a sampled row' if gen == 'anchored' else '2-6 conjuncts, random constants'}; "
                    f"estimators trained on {'/'.join(str(v) for v in train_n)} labels, {epochs} epochs",
        "note": "every mode does the same work: exact_probe0 = no mode counts the probe relation's selection "
                "(no plan depends on it), exact_probe1 = every mode counts it; capacity = the same queries "
                "offered 50x faster; predicates/s counts all three selections of every query",
        "modes": table,
        "count_errors": count_errors,
        "gate": f"beta 1.5, tau 0.05, join-order ties below selectivity {tie_cfg.tie_sel:g} (no_ties: every order "
                "counts)",
        "empty_selection_fraction": [round(v, 3) for v in empty],
        "decided_by_the_compiler_fraction": [round(v, 3) for v in decided],
        "queries_with_tied_join_order": round(ties, 3),
        "plan_agreement_with_exact": round(agree_tie, 4),
        "plan_agreement_with_exact_ties_compared": round(agree_tie_strict, 4),
        "plan_agreement_with_exact_no_ties": round(agree_strict, 4),
        "offline_training_s": round(offline_s, 1),
        "cpu_baseline": {"value": round(oracle_rows / max(oracle_s, 1e-9), 1), "unit": "row-predicates/s",
                         "cores": workers, "kind": "oracle",
                         "sample": f"{'every' if oracle_rs is None else oracle_rs} selection(s) on the 10M and 100M "
                                   f"tables, {oracle_p} on the 1B table, one process per core",
                         "checked": oracle_checked, "errors": oracle_errors, "seconds": round(oracle_s, 1)}}


def policy_workload():
    """Materialization policy on the 100M-row planning table: the cost model
    is calibrated with the library's kernels, then its keep / discard
    decisions for `lt k` selections over five decades of selectivity are
    compared with the measured cheaper option, next to a fixed threshold
    tau = 0.05 and the two trivial policies."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc, policy
    torch.cuda.init()
    ctx = esc.Context(0)
    t = dg.tables_planning([100_000_000], device="cuda:0")[0]
    dt = esc.Table(t.nrows, t.dtypes, t.cols)
    n = t.nrows
    proj, scan_cols = [1, 2], 3          # selection on column 0, columns 1 and 2 projected
    log("policy: calibration")
    model, det = policy.calibrate(ctx, dt, 0, proj, scan_cols)
    md = policy.model_dict(model)
    # measured costs per selection: re-reading the table (scan_cols columns)
    # vs the write pass plus reading the temporary table
    scratch = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    evict = lambda: scratch.sum()
    p_all = esc.Pred(dt, policy._touch_all(scan_cols))
    ws_c = ctx.workspace(dt, False, key="pol-scan")
    dcnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    scan_ms = policy._time_ms(torch, lambda: ctx.count_async(dt, p_all, dcnt, ws_c), 5, evict)
    fracs = np.logspace(-5, np.log10(0.8), 24)
    ks = [int(f * n) for f in fracs]
    ws_m = ctx.workspace(dt, True, key="pol-mat")
    cap = max(ks)
    rowids = torch.empty(cap, dtype=torch.int32, device="cuda:0")
    outs = [torch.empty(cap, dtype=torch.int32, device="cuda:0") for _ in proj]
    dmat = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    mat_ms, tmp_ms = [], []
    for k in ks:
        p = esc.Pred(dt, ("lt", 0, k))
        w = []
        for _ in range(3):
            ctx.count(dt, p, ws=ws_m)
            evict()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            ctx.materialize_async(dt, p, proj, rowids, outs, cap, dmat, ws_m)
            b.record()
            torch.cuda.synchronize()
            w.append(a.elapsed_time(b))
        assert int(dmat.item()) == k
        mat_ms.append(float(np.median(w)))
        tmp = esc.Table(k, [esc.INT32] * 3, [rowids[:k]] + [o[:k] for o in outs])
        pt = esc.Pred(tmp, policy._touch_all(3))
        ws_t = ctx.workspace(tmp, False, key=("pol-tmp", k))
        tmp_ms.append(policy._time_ms(torch, lambda: ctx.count_async(tmp, pt, dcnt, ws_t), 3, evict))
    out = {"workload": "materialization policy: 100M x 4 planning table, selection on the key, 2 projected columns",
           "model": md, "calibration": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in det.items()
                                        if k != "mat_ms"}, "by_reuses": {}}
    for r in (1, 2, 4):
        t_scan = np.full(len(ks), r * scan_ms)
        t_mat = np.asarray(mat_ms) + r * np.asarray(tmp_ms)
        best = t_mat < t_scan
        keep, _ = esc.policy_keep(model, n, np.asarray(ks, np.uint64), scan_cols, len(proj), r)
        tau, min_rows = esc.policy_thresholds(model, n, scan_cols, len(proj), r)
        pols = {"model": keep, "fixed_tau_0.05": np.asarray(fracs) < 0.05, "always": np.ones(len(ks), bool),
                "never": np.zeros(len(ks), bool)}
        opt = np.where(best, t_mat, t_scan).sum()
        res = {}
        for name, dec in pols.items():
            cost = np.where(dec, t_mat, t_scan).sum()
            res[name] = {"agreement": round(float(np.mean(dec == best)), 3),
                         "cost_ms": round(float(cost), 3), "regret_pct": round(100.0 * (cost / opt - 1.0), 2)}
        cross = [float(f) for f, a, b in zip(fracs, best[:-1], best[1:]) if a != b]
        out["by_reuses"][str(r)] = {"tau_model": round(tau, 5), "min_rows_model": round(min_rows),
                                    "measured_crossover_selectivity_above": cross[:1],
                                    "optimal_cost_ms": round(float(opt), 3), "policies": res}
    out["selectivities"] = [float(f) for f in fracs]
    out["measured_ms"] = {"scan": round(scan_ms, 4), "write": [round(v, 4) for v in mat_ms],
                          "tmp_read": [round(v, 4) for v in tmp_ms]}
    print(json.dumps(out), flush=True)


def join_workload():
    """Star join P |x| sigma(R) |x| sigma(S) after exact selectivity
    computation: the selections' exact counts order the probe's lookups (the
    more selective build side first, so most probe rows stop after one
    lookup), the selections are materialized (row id and key), hash tables
    are built on the temporary tables and the 1B-row probe relation is
    counted against both in one pass.  The reversed lookup order is timed
    beside it."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc
    torch.cuda.init()
    dev = "cuda:0"
    ctx = esc.Context(0)
    log("join: tables")
    R, S, P = dg.tables_join(device=dev)
    dR, dS = esc.Table(R.nrows, R.dtypes, R.cols), esc.Table(S.nrows, S.dtypes, S.cols)
    dP = esc.Table(P.nrows, P.dtypes, P.cols)
    queries = [(("lt", 1, 5), ("eq", 1, 0)), (("between", 1, 10, 60), ("in", 1, [1, 2, 3, 5, 8])),
               (("eq", 1, 42), ("lt", 1, 1000)), (("lt", 1, 50), ("gt", 1, 20))]
    scratch = torch.ones(1 << 28, dtype=torch.float32, device=dev)

    def timed(fn, reps=3):
        out = []
        for _ in range(reps):
            scratch.sum()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            r = fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return r, float(np.median(out))

    res = []
    sample = 20_000_000
    P_pre = esc.Table(sample, P.dtypes, [c[:sample] for c in P.cols])
    for qr, qs in queries:
        log(f"join: {qr} {qs}")
        t0 = time.perf_counter()
        sides = []
        for name, dt, q in (("R", dR, qr), ("S", dS, qs)):
            p = esc.Pred(dt, q)
            c = ctx.count(dt, p)
            ids = torch.empty(max(c, 1), dtype=torch.int32, device=dev)
            key = torch.empty(max(c, 1), dtype=torch.int32, device=dev)
            assert ctx.materialize(dt, p, [0], ids, [key], c) == c
            sides.append({"name": name, "count": c, "sel": c / dt.nrows, "key": key[:c]})
        tabs = []
        build_ms = 0.0
        for sd in sides:
            tab, ms = timed(lambda: ctx.hash_table(sd["key"]), 3)
            build_ms += ms
            tabs.append(tab)
        order = sorted(range(2), key=lambda j: sides[j]["sel"])     # the more selective side first
        cols = [0, 1]
        got, probe_ms = timed(lambda: ctx.join_count(dP, [cols[j] for j in order], [tabs[j] for j in order]))
        got_rev, probe_rev_ms = timed(lambda: ctx.join_count(dP, [cols[j] for j in order[::-1]],
                                                             [tabs[j] for j in order[::-1]]))
        assert got == got_rev
        pipeline_s = time.perf_counter() - t0
        pre = ctx.join_count(P_pre, [0, 1], tabs)
        res.append({"sel_R": round(sides[0]["sel"], 5), "sel_S": round(sides[1]["sel"], 5),
                    "build_rows": [sd["count"] for sd in sides], "join_rows": got,
                    "build_ms": round(build_ms, 3), "probe_ms": round(probe_ms, 3),
                    "probe_reversed_ms": round(probe_rev_ms, 3),
                    "order_speedup": round(probe_rev_ms / probe_ms, 2),
                    "probe_rows_per_s": round(P.nrows / (probe_ms * 1e-3), 1),
                    "probe_stream_GBps": round(P.nrows * 8 / (probe_ms * 1e-3) / 1e9, 1),
                    "pipeline_s": round(pipeline_s, 3), "prefix_rows": sample, "prefix_join_rows": pre,
                    "_keys": [sd["key"] for sd in sides]})
    # cpu_baseline: the oracle's join count over the first 20M probe rows
    from oracle import join as oj
    p_host = [c[:sample].cpu().numpy() for c in P.cols]
    errors, osec = 0, 0.0
    for r in res:
        keys = [k.cpu().numpy() for k in r.pop("_keys")]
        a = time.perf_counter()
        want = oj.count(p_host, keys)
        osec += time.perf_counter() - a
        errors += int(want != r["prefix_join_rows"])
    best = max(res, key=lambda r: r["probe_stream_GBps"])
    print(json.dumps({
        "workload": "star join: P (1B rows, 2 foreign keys) with sigma(R) (10M) and sigma(S) (100M)",
        "queries": res,
        "roofline_probe": {"bound": "hbm", "achieved": best["probe_stream_GBps"], "peak": 8000.0, "unit": "GB/s",
                           "frac": round(best["probe_stream_GBps"] / 8000.0, 4),
                           "note": "8 bytes per probe row streamed; hash lookups are extra random reads"},
        "cpu_baseline": {"value": round(len(res) * sample / osec, 1), "unit": "probe rows/s", "cores": 1,
                         "kind": "oracle", "sample": f"join count over the first {sample} probe rows, each query",
                         "errors": errors}}), flush=True)


def typed_workload(n=60_000_000, npreds=64, sample=200_000):
    """Predicates on TEXT and DECIMAL(15,2) columns (Section 3, Table 3):
    each typed predicate is lowered onto the stored int32 columns
    (dictionary codes, hundredths), compiled and counted.  Reports the
    host-side lowering + compile time per predicate, the count's rate over
    the columns it touches, and the typed oracle (strings and exact
    decimals) on a row sample as the CPU baseline, whose counts must equal
    the library's on the same sample."""
    from decimal import Decimal
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc, types
    from oracle import typed
    torch.cuda.init()
    ctx = esc.Context(0)
    log("typed: columns")
    vocab, idx, price, disc, qty = dg.typed_columns(n, dg.data_seed(7))
    wide = dg.typed_wide(n, dg.data_seed(7, 1))
    d = types.Dict(vocab)
    code_of = np.array([d.range(esc.EQ, w)[0] for w in vocab], dtype=np.int32)
    cols = [torch.from_numpy(code_of[idx]).cuda(), torch.from_numpy(price).cuda(),
            torch.from_numpy(disc).cuda(), torch.from_numpy(qty).cuda()]
    cols += [c.cuda() for c in types.split_words(torch.from_numpy(wide))]
    dt = esc.Table(n, [dg.INT32] * 6, cols)
    dt_pre = esc.Table(sample, [dg.INT32] * 6, [c[:sample] for c in cols])
    tmap = {0: ("text", d), 1: ("decimal", 2), 2: ("decimal", 2), 4: ("decimal64", 2, 5)}
    preds = dg.typed_preds(vocab, np.random.default_rng(dg.pred_seed(7)), npreds, wide=wide[:1000])
    a = time.perf_counter()
    kept, cps = [], []
    for p in preds:
        try:
            cps.append(esc.Pred(dt, types.lower(p, tmap, dt)))
            kept.append(p)
        except esc.EscError as e:      # an OR of several 64-bit decimal ranges may exceed the program limits
            if e.status != esc.ERR_UNSUPPORTED:
                raise
    lower_ms = (time.perf_counter() - a) * 1e3 / npreds
    preds = kept
    for cp in cps[:4]:
        ctx.count(dt, cp)
    torch.cuda.synchronize()
    ms, gbps, counts = [], [], []
    for p, cp in zip(preds, cps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        c = ctx.count(dt, cp)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1])
        ms.append(t)
        k = len(pred_columns(p)) + (4 in pred_columns(p))       # a 64-bit decimal reads two word columns
        gbps.append(4 * n * k / (t * 1e-3) / 1e9)
        counts.append(c)
    log("typed: oracle sample")
    text = np.array(vocab, dtype=object)[idx[:sample]]
    raw = [list(text), [Decimal(int(c)).scaleb(-2) for c in price[:sample]],
           [Decimal(int(c)).scaleb(-2) for c in disc[:sample]], qty[:sample],
           [Decimal(int(c)).scaleb(-2) for c in wide[:sample]], None]
    kinds = ["text", "decimal", "decimal", "int", "decimal", "int"]
    errors, osec, nq = 0, 0.0, 0
    for p, cp in zip(preds, cps):
        a = time.perf_counter()
        want = typed.count(raw, kinds, p)
        osec += time.perf_counter() - a
        nq += 1
        errors += int(want != ctx.count(dt_pre, cp))
        if osec > 20:
            break
    print(json.dumps({
        "workload": f"TEXT (2,000-word dictionary, Zipf 1.05) / DECIMAL(15,2) x2 in int32 / INTEGER / "
                    f"DECIMAL(15,2) in two word columns, {n} rows, {npreds} typed predicates",
        "compiled": len(cps),
        "lower_compile_ms_per_predicate": round(lower_ms, 3),
        "count_ms_p50": round(float(np.median(ms)), 4), "count_ms_max": round(float(np.max(ms)), 4),
        "count_GBps_p50": round(float(np.median(gbps)), 1),
        "selectivity_p50": round(float(np.median(counts)) / n, 5),
        "cpu_baseline": {"value": round(nq * sample / osec, 1), "unit": "rows/s", "cores": 1, "kind": "oracle",
                         "sample": f"typed oracle on the first {sample} rows, {nq} predicates",
                         "errors": errors}}), flush=True)


def sweeps_workload(n_perm=200_000_000, reps=5):
    """Synthetic analogs of the paper's selectivity and attribute-count
    measurements (Section 3, Tables 2 and 3).

    Selectivity: count(A < k) and count + materialize (row ids and A) on a
    permutation column of 2*10^8 rows for selectivities 10^-5 .. 1; every
    count must be k exactly and the materialized A values must sum to
    k(k-1)/2 (closed forms).  Attributes: conjunctions over 1..5 distinct
    columns of the 60M-row star table, counted; the counts of the first
    2*10^6 rows must equal the oracle's.  Each timing is the median of
    `reps` event-timed calls, each after a 1 GiB eviction read."""
    import torch
    from paper_1901_01488_amd import datagen as dg
    from paper_1901_01488_amd import esc
    from oracle import scan
    torch.cuda.init()
    dev = "cuda:0"
    ctx = esc.Context(0)
    scratch = torch.ones(1 << 28, dtype=torch.float32, device=dev)

    def timed(fn, fresh_ws=None):
        out, r = [], None
        for _ in range(reps):
            if fresh_ws is not None:     # forget the previous call's tiles: count again inside the timing
                esc.check(esc.lib().esc_workspace_init(ctx.h, ctypes.c_void_p(fresh_ws.data_ptr()),
                                                       fresh_ws.numel(), esc._stream_handle(None)))
            scratch.sum()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            r = fn()
            b.record()
            torch.cuda.synchronize()
            out.append(a.elapsed_time(b))
        return r, float(np.median(out))

    log("sweeps: permutation column")
    A = dg._backend(dg.data_seed(8), dev).perm(n_perm)
    dt = esc.Table(n_perm, [dg.INT32], [A])
    rowids = torch.empty(n_perm, dtype=torch.int32, device=dev)
    aout = torch.empty(n_perm, dtype=torch.int32, device=dev)
    ws = ctx.workspace(dt)                                # materialization workspace
    cws = ctx.workspace(dt, False, key="count-only")     # plain counts store no tiles
    sel_rows, errors = [], 0
    for sel in (1e-5, 1e-4, 1e-3, 1e-2, 0.1, 0.5, 1.0):
        k = int(round(sel * n_perm))
        p = esc.Pred(dt, ("lt", 0, k))
        c, t_count = timed(lambda: ctx.count(dt, p, ws=cws))
        m, t_mat = timed(lambda: ctx.materialize(dt, p, [0], rowids, [aout], n_perm, ws=ws), fresh_ws=ws)
        _, t_write = timed(lambda: ctx.materialize(dt, p, [0], rowids, [aout], n_perm, ws=ws))
        ok = c == k and m == k and int(aout[:k].to(torch.int64).sum().item()) == k * (k - 1) // 2
        errors += int(not ok)
        sel_rows.append({"selectivity": sel, "count": c, "count_ms": round(t_count, 3),
                         "count_GBps": round(4 * n_perm / (t_count * 1e-3) / 1e9, 1),
                         "count_materialize_ms": round(t_mat, 3), "materialize_after_count_ms": round(t_write, 3),
                         "materialize_out_GBps": round(8 * k / (t_mat * 1e-3) / 1e9, 1)})
    del A, rowids, aout, dt, ws, cws
    ctx._ws.clear()
    torch.cuda.empty_cache()

    log("sweeps: star table")
    t = dg.table_star(60_000_000, device=dev)
    st = esc.Table(t.nrows, t.dtypes, t.cols)
    pre_n = 2_000_000
    pre_host = dg.Table("pre", pre_n, t.dtypes, [c[:pre_n].cpu().numpy() for c in t.cols], t.kinds, t.domain)
    pre_dev = esc.Table(pre_n, t.dtypes, [c[:pre_n] for c in t.cols])
    leaves = [("between", 2, 10, 30), ("in", 3, [1, 4, 6]), ("lt", 4, np.float32(3000.0)),
              ("between", 0, dg.DATE_LO + 365, dg.DATE_LO + 1095), ("gt", 5, 150)]
    attr_rows = []
    sws = ctx.workspace(st, False, key="count-only")
    for m in range(1, 6):
        spec = leaves[0] if m == 1 else ("and", leaves[:m])
        p = esc.Pred(st, spec)
        c, tc = timed(lambda: ctx.count(st, p, ws=sws))
        errors += int(ctx.count(pre_dev, esc.Pred(pre_dev, spec)) != scan.count(pre_host, spec))
        attr_rows.append({"attributes": m, "count": c, "selectivity": round(c / t.nrows, 6),
                          "count_ms": round(tc, 3), "GBps": round(4 * m * t.nrows / (tc * 1e-3) / 1e9, 1)})
    print(json.dumps({
        "workload": "selectivity sweep on a 2*10^8-row permutation column; 1..5-attribute sweep on the "
                    "60M-row star table",
        "selectivity_sweep": sel_rows, "attribute_sweep": attr_rows, "errors": errors}), flush=True)


if __name__ == "__main__":
    main()
