"""GPU parity of the hash-join build and star-join count against the CPU
oracle: random keys with duplicates, negative and extreme values, absent
keys, empty build sides, ragged probe sizes, one to four build sides, and
the ESC pipeline (selection materialized, hash table built on its output,
probe relation counted against it)."""
import numpy as np
import pytest

from oracle import join as oj
from oracle import scan
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def _keys(rng, n, kind):
    if kind == "unique":
        return rng.permutation(n).astype(np.int32)
    if kind == "dups":
        return (rng.zipf(1.3, n) % 997).astype(np.int32)
    if kind == "neg":
        return rng.integers(-1000, 1000, n).astype(np.int32)
    return rng.choice(np.array([-2**31, 2**31 - 1, -1, 0, 1], np.int32), n)


@pytest.mark.parametrize("nprobe", [0, 1, 1023, 1025, 100_003, 2_000_001])
def test_star_join_counts(ctx, nprobe):
    rng = np.random.default_rng(100 + nprobe)
    for trial in range(6):
        k = 1 + trial % 4
        kinds = [str(rng.choice(["unique", "dups", "neg", "ext"])) for _ in range(k)]
        bsz = [int(rng.choice([0, 1, 63, 64, 1000, 100_000])) for _ in range(k)]
        builds = [_keys(rng, b, kd) for b, kd in zip(bsz, kinds)]
        probe = []
        for b, kd in zip(builds, kinds):
            pool = np.concatenate([b, rng.integers(-2000, 2000, 50).astype(np.int32)]) if len(b) else \
                rng.integers(-5, 5, 10).astype(np.int32)
            probe.append(rng.choice(pool, nprobe).astype(np.int32))
        t = esc.Table(nprobe, [esc.INT32] * k, [_dev(c) for c in probe])
        tabs = [ctx.hash_table(_dev(b)) for b in builds]
        got = ctx.join_count(t, list(range(k)), tabs)
        assert got == oj.count(probe, builds), (nprobe, kinds, bsz)


def test_table_reuse_and_rebuild(ctx):
    """A table rebuilt with other keys forgets the old ones."""
    import torch
    rng = np.random.default_rng(7)
    probe = rng.integers(0, 5000, 300_001).astype(np.int32)
    t = esc.Table(len(probe), [esc.INT32], [_dev(probe)])
    a = rng.integers(0, 2000, 1500).astype(np.int32)
    b = rng.integers(3000, 5000, 1500).astype(np.int32)
    tab = ctx.hash_table(_dev(a))
    assert ctx.join_count(t, [0], [tab]) == oj.count([probe], [a])
    import ctypes
    ka = _dev(b)
    esc.check(esc.lib().esc_hash_build(ctx.h, ctypes.c_void_p(ka.data_ptr()), len(b), ctypes.c_void_p(tab.data_ptr()),
                                       tab.numel(), None))
    assert ctx.join_count(t, [0], [tab]) == oj.count([probe], [b])
    # too small a table is refused before anything runs
    small = torch.empty(256 + 8 * 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(esc.EscError):
        esc.check(esc.lib().esc_hash_build(ctx.h, ctypes.c_void_p(ka.data_ptr()), 33, ctypes.c_void_p(small.data_ptr()),
                                           small.numel(), None))
    with pytest.raises(esc.EscError):
        ctx.join_count(t, [0], [torch.empty(1000, dtype=torch.uint8, device="cuda")])


def test_esc_pipeline_join(ctx):
    """Selections on two build relations materialized (row ids and the join
    key), hash tables built on the temporary tables, the probe relation
    counted against both: equal to the oracle's join of the filtered rows."""
    import torch
    rng = np.random.default_rng(11)
    nr, ns, npr = 200_000, 1_000_000, 3_000_017
    r_key = rng.permutation(nr).astype(np.int32)
    r_att = rng.integers(0, 100, nr).astype(np.int32)
    s_key = rng.permutation(ns).astype(np.int32)
    s_att = (rng.zipf(1.2, ns) % 1000).astype(np.int32)
    p_fr = rng.integers(0, nr, npr).astype(np.int32)
    p_fs = rng.integers(0, ns, npr).astype(np.int32)
    R = dg.Table("R", nr, [dg.INT32, dg.INT32], [r_key, r_att], ["perm", "u"], [None, None])
    S = dg.Table("S", ns, [dg.INT32, dg.INT32], [s_key, s_att], ["perm", "z"], [None, None])
    dR, dS = esc.device_table(R), esc.device_table(S)
    P = esc.Table(npr, [esc.INT32, esc.INT32], [_dev(p_fr), _dev(p_fs)])
    for sel_r, sel_s in [(("lt", 1, 7), ("in", 1, [0, 1, 5])), (("between", 1, 10, 60), ("gt", 1, 3)),
                         (("eq", 1, 1000), ("lt", 1, 1000))]:
        temps, keys_host = [], []
        for tab, dt, sel in ((R, dR, sel_r), (S, dS, sel_s)):
            p = esc.Pred(dt, sel)
            c = ctx.count(dt, p)
            ids = torch.empty(max(c, 1), dtype=torch.int32, device="cuda")
            key = torch.empty(max(c, 1), dtype=torch.int32, device="cuda")
            assert ctx.materialize(dt, p, [0], ids, [key], c) == c
            temps.append(ctx.hash_table(key[:c]))
            wc, _, wouts = scan.materialize(tab, sel, [0])
            assert wc == c
            keys_host.append(wouts[0])
        got = ctx.join_count(P, [0, 1], temps)
        assert got == oj.count([p_fr, p_fs], keys_host), (sel_r, sel_s)
