"""CPU oracle of the star-join count over hash-join build sides.

TEST INFRASTRUCTURE ONLY: used by tests and the benchmark's cpu_baseline
leg, never by the product path.

Section 2.2 probes the largest relation against hash tables built on the
other (filtered) relations.  For a probe relation P with key columns
p_1..p_K and build relations B_1..B_K with key columns b_1..b_K, the star
join P |x| B_1 |x| ... |x| B_K (on p_j = b_j) has

    sum over rows i of P of  prod_j  #{ rows r of B_j : b_j[r] = p_j[i] }

rows.  `count_loop` is that definition row by row (small inputs);
`count` evaluates it with numpy: the multiplicity of every distinct build
key, looked up for every probe key by binary search.
"""
from __future__ import annotations

from collections import Counter

import numpy as np


def count_loop(probe_cols, build_keys):
    mult = [Counter(int(k) for k in b) for b in build_keys]
    total = 0
    for i in range(len(probe_cols[0]) if probe_cols else 0):
        prod = 1
        for j, col in enumerate(probe_cols):
            prod *= mult[j].get(int(col[i]), 0)
            if prod == 0:
                break
        total += prod
    return total


def count(probe_cols, build_keys):
    n = len(probe_cols[0]) if probe_cols else 0
    prod = np.ones(n, dtype=np.uint64)
    for col, b in zip(probe_cols, build_keys):
        keys, mult = np.unique(np.asarray(b, np.int64), return_counts=True)
        c = np.asarray(col, np.int64)
        pos = np.searchsorted(keys, c)
        pos_c = np.minimum(pos, max(len(keys) - 1, 0))
        hit = (pos < len(keys)) & (keys[pos_c] == c) if len(keys) else np.zeros(n, bool)
        m = np.where(hit, mult[pos_c] if len(keys) else 0, 0).astype(np.uint64)
        prod *= m
    return int(prod.sum(dtype=np.uint64))
