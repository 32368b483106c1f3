"""Star-join count oracle against brute force and closed forms, and the
hash-table sizing of the library (host code, no GPU)."""
import ctypes
import itertools

import numpy as np
import pytest

from oracle import join as oj
from paper_1901_01488_amd import esc


def _brute(probe_cols, build_keys):
    """Nested loops over every combination of build rows."""
    total = 0
    n = len(probe_cols[0])
    for i in range(n):
        for rows in itertools.product(*[range(len(b)) for b in build_keys]):
            total += all(build_keys[j][r] == probe_cols[j][i] for j, r in enumerate(rows))
    return total


def test_count_matches_brute_force():
    rng = np.random.default_rng(1)
    for _ in range(60):
        k = int(rng.integers(1, 4))
        n = int(rng.integers(0, 12))
        probe = [rng.integers(-3, 4, n).astype(np.int32) for _ in range(k)]
        builds = [rng.integers(-3, 4, int(rng.integers(0, 6))).astype(np.int32) for _ in range(k)]
        want = _brute(probe, builds)
        assert oj.count_loop(probe, builds) == want
        assert oj.count(probe, builds) == want


def test_closed_forms():
    rng = np.random.default_rng(2)
    # primary-key build side: each probe key in [0, m) matches exactly once
    m = 1000
    probe = rng.integers(-50, m + 50, 20000).astype(np.int32)
    assert oj.count([probe], [rng.permutation(m).astype(np.int32)]) == int(((probe >= 0) & (probe < m)).sum())
    # one key everywhere: every probe row pairs with every build row
    p = [np.full(17, 5, np.int32), np.full(17, -9, np.int32)]
    b = [np.full(4, 5, np.int32), np.full(6, -9, np.int32)]
    assert oj.count(p, b) == 17 * 4 * 6 == oj.count_loop(p, b)
    # an empty build side empties the join
    assert oj.count([probe], [np.zeros(0, np.int32)]) == 0
    # int32 extremes are ordinary keys
    ext = np.array([-2**31, 2**31 - 1, 0, -1], np.int32)
    assert oj.count([ext], [np.array([-2**31, -2**31, -1], np.int32)]) == 3
    # multiplicities multiply across build sides
    p = [np.array([1, 2, 3], np.int32), np.array([7, 7, 8], np.int32)]
    b = [np.array([1, 1, 2, 3, 3, 3], np.int32), np.array([7, 7, 7, 8], np.int32)]
    assert oj.count(p, b) == 2 * 3 + 1 * 3 + 3 * 1


def test_hash_table_sizes():
    L = esc.lib()
    nb = ctypes.c_size_t()
    for n, slots in [(0, 64), (1, 64), (32, 64), (33, 128), (1000, 2048), (1 << 20, 1 << 21)]:
        assert L.esc_hash_table_bytes(n, ctypes.byref(nb)) == esc.OK
        assert nb.value == 256 + 8 * slots
    assert L.esc_hash_table_bytes(-1, ctypes.byref(nb)) == esc.ERR_INVALID
    assert L.esc_hash_table_bytes((1 << 30) + 1, ctypes.byref(nb)) == esc.ERR_UNSUPPORTED
