"""GPU parity of TEXT and DECIMAL predicates (Section 3, Table 3).

The typed predicates are lowered onto the stored int32 columns (dictionary
codes, hundredths) and run through esc_count / esc_materialize; counts and
row ids must equal the typed oracle's, which compares the strings and exact
decimals themselves."""
from decimal import Decimal

import numpy as np
import pytest

from oracle import typed
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc, types

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def workload(n, seed):
    vocab, idx, price, disc, qty = dg.typed_columns(n, seed)
    text = np.array(vocab, dtype=object)[idx]
    raw = [list(text), [Decimal(int(c)).scaleb(-2) for c in price],
           [Decimal(int(c)).scaleb(-2) for c in disc], qty]
    d = types.Dict(vocab)
    t = dg.Table("typed", n, [dg.INT32] * 4, [d.encode(text), price, disc, qty], ["text", "dec", "dec", "int"],
                 [None] * 4)
    return vocab, raw, t, {0: ("text", d), 1: ("decimal", 2), 2: ("decimal", 2)}


KINDS = ["text", "decimal", "decimal", "int"]


@pytest.mark.parametrize("n,seed,npreds", [(0, 31, 10), (1, 32, 20), (4097, 33, 40), (100_003, 34, 60)])
def test_typed_counts_and_rows(ctx, n, seed, npreds):
    import torch
    vocab, raw, t, tmap = workload(n, seed)
    dt = esc.device_table(t)
    preds = dg.typed_preds(vocab, np.random.default_rng(seed + 100), npreds)
    for i, p in enumerate(preds):
        want = np.flatnonzero(typed.eval_rows(raw, KINDS, p)) if n else np.zeros(0, np.int64)
        cp = esc.Pred(dt, types.lower(p, tmap))
        got = ctx.count(dt, cp)
        assert got == len(want), (n, i, p)
        if i % 4 == 0:
            cap = max(got, 1)
            rowids = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
            outs = [torch.zeros(cap, dtype=torch.int32, device="cuda")]
            c = ctx.materialize(dt, cp, [0], rowids, outs, got)
            assert c == got
            ids = rowids[:got].cpu().numpy()
            assert np.array_equal(ids, want), (n, i, p)
            assert np.array_equal(outs[0][:got].cpu().numpy(), t.cols[0][want])
