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
    """Columns: TEXT codes, DECIMAL(15,2) price and discount in int32,
    INTEGER quantity, and a DECIMAL(15,2) column beyond int32 as its two
    word columns 4 (H) and 5 (L)."""
    vocab, idx, price, disc, qty = dg.typed_columns(n, seed)
    wide = dg.typed_wide(n, seed + 7)
    text = np.array(vocab, dtype=object)[idx]
    raw = [list(text), [Decimal(int(c)).scaleb(-2) for c in price],
           [Decimal(int(c)).scaleb(-2) for c in disc], qty, [Decimal(int(c)).scaleb(-2) for c in wide], None]
    d = types.Dict(vocab)
    hi, lo = types.split_words(wide)
    t = dg.Table("typed", n, [dg.INT32] * 6, [d.encode(text), price, disc, qty, hi, lo],
                 ["text", "dec", "dec", "int", "dec64 hi", "dec64 lo"], [None] * 6)
    return vocab, wide, raw, t, {0: ("text", d), 1: ("decimal", 2), 2: ("decimal", 2), 4: ("decimal64", 2, 5)}


KINDS = ["text", "decimal", "decimal", "int", "decimal", "int"]


@pytest.mark.parametrize("n,seed,npreds", [(0, 31, 10), (1, 32, 20), (4097, 33, 40), (100_003, 34, 60)])
def test_typed_counts_and_rows(ctx, n, seed, npreds):
    import torch
    vocab, wide, raw, t, tmap = workload(n, seed)
    dt = esc.device_table(t)
    sample = wide[:1000] if n else dg.typed_wide(1000, seed)
    preds = dg.typed_preds(vocab, np.random.default_rng(seed + 100), npreds, wide=sample)
    unsupported = 0
    for i, p in enumerate(preds):
        want = np.flatnonzero(typed.eval_rows(raw, KINDS, p)) if n else np.zeros(0, np.int64)
        try:
            cp = esc.Pred(dt, types.lower(p, tmap, dt))
        except esc.EscError as e:     # rare ORs of several 64-bit decimal ranges exceed the program limits
            assert e.status == esc.ERR_UNSUPPORTED, (e, p)
            unsupported += 1
            continue
        got = ctx.count(dt, cp)
        assert got == len(want), (n, i, p)
        if i % 4 == 0:
            cap = max(got, 1)
            rowids = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
            outs = [torch.zeros(cap, dtype=torch.int32, device="cuda") for _ in range(3)]
            c = ctx.materialize(dt, cp, [0, 4, 5], rowids, outs, got)
            assert c == got
            ids = rowids[:got].cpu().numpy()
            assert np.array_equal(ids, want), (n, i, p)
            assert np.array_equal(outs[0][:got].cpu().numpy(), t.cols[0][want])
            # the 64-bit decimal, rebuilt from its two projected word columns
            hi = outs[1][:got].cpu().numpy().astype(np.int64)
            lo = outs[2][:got].cpu().numpy().view(np.uint32).astype(np.int64) ^ 0x80000000
            assert np.array_equal(hi * 2**32 + lo, wide[want]), (n, i, p)
    assert unsupported <= max(1, npreds // 20)
