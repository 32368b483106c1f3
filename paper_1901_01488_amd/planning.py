"""Planning-time workload: arriving three-table join queries whose selection
cardinalities are decided by exact selectivity computation, plain or batched,
with or without the learned gate.

Each query has one selection per table: two build relations R and S and the
largest relation P, which is probed (Section 2.2: hash tables are built on
all but the largest relation).  The optimizer needs, per query:
  - push-down of each build-side selection: only when its selectivity is
    below the maximum threshold tau and the table has more than min_rows
    rows (Section 2.1);
  - join order: the smaller filtered build relation first (Section 2.2);
    both orders cost the same when each build relation keeps at most
    tie_sel of its rows (the relation joined first passes sel * |P| probe
    rows on to the second lookup), so the order is then left open;
  - no push-down on the probe relation (Section 2.2), so its cardinality
    does not change the plan.
Every mode takes `exact_probe`: with it off, no mode counts the probe
relation's selection (the plan does not depend on it); with it on, every
mode counts it.  Modes are thus compared on identical work.  Latency of a
query is the time from its arrival until its selectivities are decided.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import esc


@dataclass
class GateConfig:
    tau: float = 0.05
    min_rows: int = 1_000_000
    beta: float = 1.25
    exact_probe: bool = False
    tie_sel: float = 1e-3   # 0: every join order counts, however small both relations are


def decide(sel_r, sel_s, n_r, n_s, g: GateConfig):
    """Plan decisions from (estimated or exact) selectivities of R and S."""
    push_r = n_r >= g.min_rows and sel_r < g.tau
    push_s = n_s >= g.min_rows and sel_s < g.tau
    r_first = sel_r * n_r <= sel_s * n_s
    return push_r, push_s, r_first


def agree(exact, other, sel_exact, g: GateConfig):
    """Whether a plan is as good as the exact one: the same push-down
    decisions and the same join order, unless both build relations of the
    exact plan keep at most tie_sel of their rows (then both orders cost
    the same)."""
    tie = g.tie_sel > 0.0 and sel_exact[0] <= g.tie_sel and sel_exact[1] <= g.tie_sel
    return exact[0] == other[0] and exact[1] == other[1] and (tie or exact[2] == other[2])


class Workload:
    def __init__(self, ctx, tables, queries, arrivals):
        """tables: [R, S, P] esc.Table (device); queries: list of 3-tuples of
        predicate descriptions; arrivals: seconds, increasing."""
        self.ctx = ctx
        self.tables = tables
        self.queries = queries
        self.arrivals = np.asarray(arrivals, np.float64)
        self.cps = [[esc.Pred(tables[t], q[t]) for t in range(3)] for q in queries]
        # counts the compiler already decided (contradictory conjuncts: 0;
        # always true: the table's rows), -1 where a scan is needed
        self.known = np.full((len(queries), 3), -1, np.int64)
        for i, row in enumerate(self.cps):
            for t, cp in enumerate(row):
                c = cp.info()["constant"]
                if c != 0:
                    self.known[i, t] = tables[t].nrows if c > 0 else 0
        self.ws = [ctx.workspace(t, False, key=("plan", i)) for i, t in enumerate(tables)]
        self.batch = None   # one batched handle, re-planned per micro-batch

    # --------------------------------------------------------- plain
    def run_plain(self, exact_probe=True):
        """Queries in arrival order; each needed selectivity by one esc_count."""
        tabs = range(3) if exact_probe else range(2)
        n = len(self.queries)
        done = np.zeros(n)
        counts = np.zeros((n, 3), np.uint64)
        t0 = time.perf_counter()
        for i in range(n):
            now = time.perf_counter() - t0
            if now < self.arrivals[i]:
                time.sleep(self.arrivals[i] - now)
            for t in tabs:
                counts[i, t] = self.ctx.count(self.tables[t], self.cps[i][t], ws=self.ws[t])
            done[i] = time.perf_counter() - t0
        return self._report(done, counts, 3 * n, "plain")

    # --------------------------------------------------------- batched (+ gate)
    def run_batched(self, window=64, max_wait_s=1e-3, gate=None, estimators=None, gcfg: GateConfig = None,
                    exact_probe=True):
        """Micro-batches of arriving queries: when `window` queries are
        pending or the oldest has waited max_wait_s, the pending selections
        go to one batched graph launch.  With a gate, each pending selection
        is first estimated and only the routed ones are counted exactly (the
        gate's exact_probe decides for the probe relation)."""
        if gcfg is not None:
            exact_probe = gcfg.exact_probe
        ntabs = 3 if exact_probe else 2
        n = len(self.queries)
        done = np.zeros(n)
        counts = np.zeros((n, 3), np.uint64)
        est = np.full((n, 3), np.nan)
        routed = np.zeros((n, 3), bool)
        nrows = [t.nrows for t in self.tables]
        t0 = time.perf_counter()
        i = 0
        exact_preds = 0
        while i < n:
            now = time.perf_counter() - t0
            if now < self.arrivals[i]:
                time.sleep(self.arrivals[i] - now)
                now = time.perf_counter() - t0
            # pending = arrived queries from i on, up to `window`
            j = i
            while j < n and j - i < window and self.arrivals[j] <= now:
                j += 1
            if j - i < window and j < n:
                # wait for more arrivals until the oldest has waited max_wait_s
                deadline = self.arrivals[i] + max_wait_s
                while j < n and j - i < window and self.arrivals[j] <= deadline:
                    if now < self.arrivals[j]:
                        time.sleep(max(0.0, min(self.arrivals[j], deadline) - now))
                        now = time.perf_counter() - t0
                    if self.arrivals[j] <= now:
                        j += 1
                    else:
                        break
                if now < deadline and j - i < window:
                    time.sleep(max(0.0, deadline - now))
                    now = time.perf_counter() - t0
                    while j < n and j - i < window and self.arrivals[j] <= now:
                        j += 1
            need = [(q, t) for q in range(i, j) for t in range(ntabs)]
            if gate is not None:
                need = []
                # the build relations' selections are estimated (those whose
                # count the compiler decided are exact already: their
                # "estimate" is that count); no plan decision reads the
                # probe relation's (it is counted or not according to
                # exact_probe, as in the other modes)
                for t in range(2):
                    kn = self.known[i:j, t]
                    todo = [q for q in range(i, j) if kn[q - i] < 0]
                    yh = np.log(np.maximum(kn, 1) / float(nrows[t])).astype(np.float32)
                    if todo:
                        x = estimators[t].features([self.cps[q][t] for q in todo])
                        yh[np.array(todo) - i] = estimators[t].predict(x)
                    est[i:j, t] = yh
                    routed[i:j, t] |= esc.gate_pushdown(yh, nrows[t], gcfg.tau, gcfg.beta, gcfg.min_rows) & (kn < 0)
                routed[i:j, 2] = gcfg.exact_probe
                pair = esc.gate_join_pairs(est[i:j, 0], nrows[0], est[i:j, 1], nrows[1], gcfg.beta, gcfg.tie_sel)
                routed[i:j, 0] |= pair & (self.known[i:j, 0] < 0)
                routed[i:j, 1] |= pair & (self.known[i:j, 1] < 0)
                kn_all = self.known[i:j]
                counts[i:j][kn_all >= 0] = kn_all[kn_all >= 0].astype(np.uint64)
                need = [(q, t) for q in range(i, j) for t in range(3) if routed[q, t]]
            if need:
                preds = [self.cps[q][t] for q, t in need]
                owners = [t for _, t in need]
                if self.batch is None:
                    # 16 rows per lane, groups of 16 predicates, the
                    # kernel with four column slots (the tables have four
                    # columns): the fastest measured for these windows
                    self.batch = esc.Batch(self.ctx, self.tables, preds, owners, rows_per_thread=16, group=16,
                                           max_preds=3 * window)
                else:
                    self.batch.update(preds, owners)
                c = self.batch.count()
                for (q, t), v in zip(need, c):
                    counts[q, t] = v
                exact_preds += len(need)
            done[i:j] = time.perf_counter() - t0
            i = j
        rep = self._report(done, counts, 3 * n, "batched" if gate is None else "batched+gate")
        rep["exact_fraction"] = exact_preds / (3.0 * n)
        rep["est"] = est
        rep["routed"] = routed
        rep["known"] = self.known >= 0   # counts the compiler decided (exact, no scan)
        return rep

    def _report(self, done, counts, npreds, name):
        lat = (done - self.arrivals) * 1e3
        makespan = float(done[-1] - 0.0) if len(done) else 0.0
        return {"mode": name, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "predicates_per_s": npreds / max(makespan - float(self.arrivals[0]), 1e-9),
                "makespan_s": makespan, "counts": counts}


def plans(sel, nrows, gcfg):
    """Plan decisions of every query from a (n, 3) selectivity array."""
    out = []
    for s in sel:
        out.append(decide(s[0], s[1], nrows[0], nrows[1], gcfg))
    return out
