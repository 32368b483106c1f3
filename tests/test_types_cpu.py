"""TEXT and DECIMAL predicates (Section 3, Table 3) on the host.

The dictionary ranges and decimal bounds of the library are checked against
brute force over the strings and against Python's exact decimal arithmetic;
the typed oracle is pinned on hand-worked cases; and the lowering of typed
predicates onto the stored int32 columns is checked end to end against the
typed oracle by counting the lowered predicates with the scan oracle."""
from decimal import Decimal

import os

import numpy as np
import pytest

from oracle import scan, typed
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc, types


def b(s):
    return s.encode()


# ---------------------------------------------------------------- typed oracle pins

def test_typed_oracle_hand_cases():
    text = ["apple", "apricot", "b", "banana", "", "Apple", "äpfel"]
    dec = [Decimal("0.10"), Decimal("0.05"), Decimal("-1.00"), Decimal("12.34"),
           Decimal("0.00"), Decimal("0.05"), Decimal("99.99")]
    cols, kinds = [text, dec], ["text", "decimal"]
    cases = [
        (("prefix", 0, "ap"), [0, 1]),
        (("prefix", 0, ""), [0, 1, 2, 3, 4, 5, 6]),
        (("lt", 0, "b"), [0, 1, 4, 5]),             # "" and "Apple" (uppercase sorts first)
        (("gt", 0, "b"), [3, 6]),                   # "banana" and "ä" (code point 228)
        (("between", 0, "apricot", "banana"), [1, 2, 3]),
        (("eq", 0, "applE"), []),
        (("in", 0, ["b", "zz", ""]), [2, 4]),
        (("eq", 1, "0.05"), [1, 5]),
        (("eq", 1, "0.050"), [1, 5]),
        (("eq", 1, "0.055"), []),
        (("lt", 1, "0.055"), [1, 2, 4, 5]),
        (("gt", 1, "0.099"), [0, 3, 6]),
        (("between", 1, "-1", "0.05"), [1, 2, 4, 5]),
        (("in", 1, ["12.340", "-1", "7"]), [2, 3]),
        (("and", [("prefix", 0, "a"), ("gt", 1, "0.07")]), [0]),
        (("or", [("eq", 0, "b"), ("lt", 1, "0")]), [2]),
    ]
    for pred, rows in cases:
        assert list(np.flatnonzero(typed.eval_rows(cols, kinds, pred))) == rows, pred


# ---------------------------------------------------------------- dictionary

@pytest.fixture(scope="module")
def vocab():
    return dg.typed_vocab(300, 11)


def test_dict_order_and_codes(vocab):
    d = types.Dict(vocab)
    assert d.strings == sorted(vocab, key=b)
    for c, s in enumerate(d.strings):
        assert d.range(esc.EQ, s) == (c, c)
    assert d.range(esc.EQ, "not-in-it") == (0, -1)
    assert list(d.encode(d.strings)) == list(range(len(vocab)))


def test_dict_rejects_duplicates():
    with pytest.raises(esc.EscError):
        types.Dict(["a", "b", "a"])


def test_nul_is_refused():
    with pytest.raises(ValueError):
        types.Dict(["a\x00b"])
    with pytest.raises(ValueError):
        types.Dict(["a"]).range(esc.EQ, "a\x00")


def test_empty_dict():
    d = types.Dict([])
    for op in (esc.EQ, esc.LT, esc.GT, esc.DICT_PREFIX):
        assert d.range(op, "x") == (0, -1)


def test_dict_ranges_brute_force(vocab):
    d = types.Dict(vocab)
    bs = [b(s) for s in d.strings]
    rng = np.random.default_rng(3)
    probes = list(vocab[:60]) + [s + "m" for s in vocab[:20]] + [s[:2] for s in vocab[:30]] + \
        ["", "~", "\U0001f600", "zzzzzzzzzzzzz", "a", "b\x01"]
    for s in probes:
        t = rng.choice(probes)
        want = {
            esc.EQ: [c for c, x in enumerate(bs) if x == b(s)],
            esc.LT: [c for c, x in enumerate(bs) if x < b(s)],
            esc.GT: [c for c, x in enumerate(bs) if x > b(s)],
            esc.BETWEEN: [c for c, x in enumerate(bs) if b(s) <= x <= b(t)],
            esc.DICT_PREFIX: [c for c, x in enumerate(bs) if x.startswith(b(s))],
        }
        for op, rows in want.items():
            lo, hi = d.range(op, s, t if op == esc.BETWEEN else None)
            assert list(range(lo, hi + 1)) == rows, (op, s, t)


# ---------------------------------------------------------------- decimal bounds

def _literals(rng, k):
    out = ["0", "-0", "0.00", "-0.001", "+5", ".5", "5.", "0.005", "-0.005", "21474836.47",
           "21474836.48", "-21474836.48", "123456789012345.99", "999999999999999999", "1.000000001"]
    for _ in range(k):
        ip = str(int(rng.integers(0, 10 ** int(rng.integers(1, 10)))))
        fp = "".join(rng.choice(list("0123456789"), int(rng.integers(0, 6))))
        sign = ["", "-", "+"][rng.integers(3)]
        out.append(sign + ip + ("." + fp if fp or rng.random() < 0.1 else ""))
    return out


@pytest.mark.parametrize("scale", [0, 2, 5, 9])
def test_decimal_bounds_exact(scale):
    rng = np.random.default_rng(scale)
    for lit in _literals(rng, 300):
        v = Decimal(lit).scaleb(scale)      # the literal in stored units, exact
        if abs(v) >= 10 ** 18:
            continue                        # saturates (test_decimal_bound_errors)
        e, empty = types.decimal_bound(lit, scale, esc.EQ)
        assert empty == (v != v.to_integral_value()), lit
        if not empty:
            assert e == int(v), lit
        lt = types.decimal_bound(lit, scale, esc.LT)[0]
        assert lt < v and lt + 1 >= v, lit        # the largest stored value below v
        gt = types.decimal_bound(lit, scale, esc.GT)[0]
        assert gt > v and gt - 1 <= v, lit        # the smallest stored value above v


def test_decimal_bound_errors():
    for lit in ["", "+", "-", ".", "1e5", "1.2.3", " 1", "1 ", "0x10", "nan"]:
        with pytest.raises(esc.EscError) as ei:
            types.decimal_bound(lit, 2, esc.EQ)
        assert ei.value.status == esc.ERR_INVALID, lit
    with pytest.raises(esc.EscError):
        types.decimal_bound("1", 10, esc.EQ)
    assert types.decimal_bound("9" * 18, 0, esc.EQ) == (int("9" * 18), False)
    # 10^18 and beyond saturate to +-(10^18 + 1/2)
    big = 10 ** 18
    for lit, sc in [("1" + "0" * 18, 0), ("1" * 19, 0), ("12345678901234567.89", 2), ("9" * 40 + ".5", 0)]:
        assert types.decimal_bound(lit, sc, esc.EQ)[1]
        assert types.decimal_bound(lit, sc, esc.LT)[0] == big
        assert types.decimal_bound(lit, sc, esc.GT)[0] == big + 1
        assert types.decimal_bound("-" + lit, sc, esc.LT)[0] == -big - 1
        assert types.decimal_bound("-" + lit, sc, esc.GT)[0] == -big


# ---------------------------------------------------------------- lowering, end to end on the CPU

def test_word_split_order():
    x = np.array(sorted(set(dg.WIDE_EDGES + [-2**63, 2**63 - 1, 5, -5, 2**40 + 3])), dtype=np.int64)
    hi, lo = types.split_words(x)
    assert np.array_equal(np.lexsort((lo, hi)), np.arange(len(x)))   # (H, L) order = value order
    assert np.array_equal(hi.astype(np.int64) * 2**32 + (lo.view(np.uint32) ^ 0x80000000), x)


def test_range64_brute_force():
    """Every 64-bit range between word-edge bounds (and open ends), lowered by
    the library onto the two word columns (a DECIMAL(18,0) column, so each
    literal is its stored value), against numpy's int64 comparison."""
    edges = sorted({e + d for e in dg.WIDE_EDGES for d in (-1, 0, 1)} | {-7 * 2**32 + 5, 3 * 2**32})
    x = np.array(edges, dtype=np.int64)
    hi, lo = types.split_words(x)
    t = dg.Table("w", len(x), [dg.INT32] * 2, [hi, lo], ["h", "l"], [None] * 2)
    tmap = {0: ("decimal64", 0, 1)}
    bounds = edges[::2] + [None]
    for a in bounds:
        for c in bounds:
            want = np.ones(len(x), bool)
            if a is not None:
                want &= x >= a
            if c is not None:
                want &= x <= c
            if a is not None and c is not None:
                p = ("between", 0, str(a), str(c))
            elif a is not None:
                p = ("gt", 0, str(a - 1))          # x > a - 1 <=> x >= a for integers
            elif c is not None:
                p = ("lt", 0, str(c + 1))
            else:
                continue
            got = scan.eval_rows(t, types.lower(p, tmap, t.dtypes)).astype(bool)
            assert np.array_equal(got, want), (a, c)


def test_lowering_errors_and_capacity():
    """The library refuses a prefix match on a DECIMAL column, a typed
    column not stored as int32 and a malformed literal, and reports the
    sizes a too-small output needs."""
    d = types.Dict(["a", "b"])
    with pytest.raises(esc.EscError) as e:
        types.lower(("prefix", 1, "1"), {0: ("text", d), 1: ("decimal", 2)}, [dg.INT32, dg.INT32])
    assert e.value.status == esc.ERR_TYPE
    with pytest.raises(esc.EscError) as e:
        types.lower(("eq", 0, "1.5"), {0: ("decimal", 2)}, [dg.FLOAT32])
    assert e.value.status == esc.ERR_TYPE
    with pytest.raises(esc.EscError) as e:
        types.lower(("eq", 0, "1.2.3"), {0: ("decimal", 2)}, [dg.INT32])
    assert e.value.status == esc.ERR_INVALID
    # an IN of many wide values grows the tree beyond the first guess of its size
    vals = [str(v) for v in range(0, 2**32 * 40, 2**32 + 7)]
    low = types.lower(("in", 0, vals), {0: ("decimal64", 0, 1)}, [dg.INT32, dg.INT32])
    assert low[0] == "and" and len(low[1]) == 1 + len(vals)


def typed_workload(n, seed):
    vocab, idx, price, disc, qty = dg.typed_columns(n, seed)
    wide = dg.typed_wide(n, seed + 7)
    text = np.array(vocab, dtype=object)[idx]
    raw = [list(text), [Decimal(int(c)).scaleb(-2) for c in price],
           [Decimal(int(c)).scaleb(-2) for c in disc], qty, [Decimal(int(c)).scaleb(-2) for c in wide], None]
    kinds = ["text", "decimal", "decimal", "int", "decimal", "int"]
    return vocab, idx, price, disc, qty, wide, raw, kinds


def lowered_table(vocab, idx, price, disc, qty, wide):
    d = types.Dict(vocab)
    codes = d.encode(np.array(vocab, dtype=object)[idx])
    hi, lo = types.split_words(wide)
    t = dg.Table("typed", len(idx), [dg.INT32] * 6, [codes, price, disc, qty, hi, lo],
                 ["text", "dec", "dec", "int", "dec64 hi", "dec64 lo"], [None] * 6)
    return d, t


def test_lowered_counts_match_typed_oracle():
    vocab, idx, price, disc, qty, wide, raw, kinds = typed_workload(20_000, 21)
    d, t = lowered_table(vocab, idx, price, disc, qty, wide)
    tmap = {0: ("text", d), 1: ("decimal", 2), 2: ("decimal", 2), 4: ("decimal64", 2, 5)}
    preds = dg.typed_preds(vocab, np.random.default_rng(22), 200, wide=wide[:1000])
    nonzero = 0
    for p in preds:
        want = typed.eval_rows(raw, kinds, p)
        got = scan.eval_rows(t, types.lower(p, tmap, t.dtypes))
        assert np.array_equal(got.astype(bool), want), p
        nonzero += 0 < want.sum() < len(want)
    assert nonzero > 40      # the workload is not degenerate


def test_lowered_predicates_compile():
    """The lowered typed workload fits the compiled program limits, apart
    from rare ORs of several 64-bit decimal ranges (each a few clauses, and
    an OR distributes them)."""
    vocab, idx, price, disc, qty, wide, raw, kinds = typed_workload(2000, 21)
    d, t = lowered_table(vocab, idx, price, disc, qty, wide)
    tmap = {0: ("text", d), 1: ("decimal", 2), 2: ("decimal", 2), 4: ("decimal64", 2, 5)}
    st = esc.schema_table(t)
    unsupported = 0
    preds = dg.typed_preds(vocab, np.random.default_rng(23), 400, wide=wide[:1000])
    for p in preds:
        try:
            esc.Pred(st, types.lower(p, tmap, t.dtypes))
        except esc.EscError as e:
            assert e.status == esc.ERR_UNSUPPORTED, (e, p)
            unsupported += 1
    assert unsupported <= len(preds) // 100


def test_lowering_edge_cases():
    """Empty and degenerate typed leaves lower to exact int32 leaves."""
    d = types.Dict(["b", "ba", "c"])
    text = ["b", "ba", "c", "ba", "b"]
    dec = [Decimal("1.00"), Decimal("-2.50"), Decimal("0.01"), Decimal("1.00"), Decimal("21474836.47")]
    wide = [10**15 - 1, -(10**15 - 1), 2**32, 0, -1]
    hi, lo = types.split_words(np.array(wide, dtype=np.int64))
    raw = [text, dec, [Decimal(w).scaleb(-2) for w in wide], None]
    kinds = ["text", "decimal", "decimal", "int"]
    t = dg.Table("e", 5, [dg.INT32] * 4, [d.encode(text), np.array([100, -250, 1, 100, 2**31 - 1], np.int32), hi, lo],
                 ["t", "d", "h", "l"], [None] * 4)
    tmap = {0: ("text", d), 1: ("decimal", 2), 2: ("decimal64", 2, 3)}
    cases = [
        ("prefix", 0, ""), ("prefix", 0, "b"), ("prefix", 0, "bb"), ("in", 0, ["zz", "a"]), ("in", 0, ["c", "c"]),
        ("between", 0, "c", "b"), ("lt", 0, ""), ("gt", 0, "c"), ("eq", 0, "ba"),
        ("between", 1, "2", "1"), ("in", 1, ["1.001", "7"]), ("in", 1, ["1", "0.010"]), ("eq", 1, "21474836.47"),
        ("gt", 1, "21474836.47"), ("lt", 1, "-99999999999"), ("gt", 1, "-99999999999.5"),
        ("eq", 2, "9999999999999.99"), ("lt", 2, "-9999999999999.99"), ("between", 2, "-0.01", "42949672.96"),
        ("in", 2, ["42949672.96", "-0.01", "0", "3.333"]), ("gt", 2, "1e3".replace("e3", "000")),
        ("or", [("prefix", 0, "b"), ("eq", 2, "0")]), ("and", [("gt", 1, "0"), ("lt", 2, "1")]),
    ]
    for p in cases:
        want = typed.eval_rows(raw, kinds, p)
        got = scan.eval_rows(t, types.lower(p, tmap, t.dtypes)).astype(bool)
        assert np.array_equal(got, want), p


def test_c_caller_lowers_a_wide_decimal_predicate(tmp_path):
    """tests/c/lower_typed.c, built with gcc against include/esc.h and the
    built libesc.so, lowers and compiles a 64-bit DECIMAL range and a TEXT
    prefix through the C ABI alone."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    lib_dir = os.path.dirname(esc.LIB_PATH)
    exe = tmp_path / "lower_typed"
    subprocess.run(["gcc", "-std=c11", "-O1", "-Wall", "-I", os.path.join(root, "include"),
                    os.path.join(root, "tests", "c", "lower_typed.c"), "-o", str(exe), "-L", lib_dir, "-lesc",
                    "-Wl,-rpath," + lib_dir], check=True, capture_output=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
