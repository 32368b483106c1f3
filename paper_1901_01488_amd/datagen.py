"""Seeded synthetic inputs for exact selectivity computation.

This module only *draws* inputs: columnar tables and predicate descriptions.
It holds none of the method's arithmetic (no predicate evaluation, no
counting), so both the GPU path and the CPU oracle may be fed from it.

The paper measures on TPC-H (scale factors 1/10/50) and SSB (scale factor 80)
with one selection per table (Section 3).  Those datasets are not used here;
the tables below are synthetic stand-ins with the shapes that matter for a
selection scan: uniform, skewed (bounded Zipf), correlated and float columns,
a permutation key, and star-schema style fact tables.

Predicate description format (nested tuples, shared by all consumers):

    P := ("and", [P, ...]) | ("or", [P, ...])
       | ("eq", c, k) | ("lt", c, k) | ("gt", c, k)
       | ("between", c, lo, hi) | ("in", c, [k, ...])
       | ("udf", E, T)
    T := ("eq", k) | ("lt", k) | ("gt", k) | ("between", lo, hi) | ("in", [k, ...])
    E := ("col", c) | ("const", k) | (op, E, ("col", c) | ("const", k))
         op in add sub mul mod band bor bxor shl shr   (left-deep chains)

Constants on int32/date32 columns and in udfs are Python ints; constants on
float32 columns are numpy.float32 values.

Two backends draw columns: numpy PCG64 (``default_rng``) for tables that the
host must hold anyway, and torch generators on a device for the large tables
(10^8..10^9 rows) that only need host samples.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

INT32, DATE32, FLOAT32 = 0, 1, 2
DTYPE_NAMES = {INT32: "int32", DATE32: "date32", FLOAT32: "float32"}

# 1992-01-01 as int32 days since 1970-01-01, and a 7-year (2,557-day) span
DATE_LO = 8035
DATE_SPAN = 2557

# seeds: data 1901 + 1000*config + table, predicates 1488 + 1000*config, MLP 7
def data_seed(config: int, table: int = 0) -> int:
    return 1901 + 1000 * config + table


def pred_seed(config: int) -> int:
    return 1488 + 1000 * config


MLP_SEED = 7


@dataclass
class Table:
    """A columnar table: equal-length 1-D arrays (numpy or torch), 4 bytes each."""
    name: str
    nrows: int
    dtypes: list
    cols: list
    kinds: list = field(default_factory=list)   # generator kind of each column
    domain: list = field(default_factory=list)  # (lo, hi) inclusive domain, ints; None for floats

    def host(self) -> "Table":
        cols = [c if isinstance(c, np.ndarray) else c.cpu().numpy() for c in self.cols]
        return Table(self.name, self.nrows, list(self.dtypes), cols, list(self.kinds), list(self.domain))


# ---------------------------------------------------------------- columns

class _NumpyBackend:
    def __init__(self, seed):
        self.rng = np.random.default_rng(seed)

    def perm(self, n):
        return self.rng.permutation(n).astype(np.int32)

    def uniform(self, lo, hi, n):  # [lo, hi)
        return self.rng.integers(lo, hi, n, dtype=np.int64).astype(np.int32)

    def zipf(self, s, k, n):
        cdf = _zipf_cdf(s, k)
        u = self.rng.random(n)
        v = np.searchsorted(cdf, u, side="right")
        return np.minimum(v, k - 1).astype(np.int32)

    def lognormal_f32(self, mu, sigma, n):
        z = self.rng.standard_normal(n)
        return np.exp(mu + sigma * z).astype(np.float32)

    def add(self, a, b):
        return (a.astype(np.int64) + b).astype(np.int32)

    def scale(self, a, m):
        return (a.astype(np.int64) * m).astype(np.int32)


class _TorchBackend:
    def __init__(self, seed, device):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.g = torch.Generator(device=self.dev)
        self.g.manual_seed(seed)

    def perm(self, n):
        return self.torch.randperm(n, generator=self.g, device=self.dev, dtype=self.torch.int64).to(self.torch.int32)

    def uniform(self, lo, hi, n):
        return self.torch.randint(lo, hi, (n,), generator=self.g, device=self.dev, dtype=self.torch.int32)

    def zipf(self, s, k, n):
        t = self.torch
        cdf = t.from_numpy(_zipf_cdf(s, k)).to(self.dev)
        out = t.empty(n, dtype=t.int32, device=self.dev)
        step = 1 << 26
        for i in range(0, n, step):
            m = min(step, n - i)
            u = t.rand(m, generator=self.g, device=self.dev, dtype=t.float64)
            v = t.searchsorted(cdf, u, right=True)
            out[i:i + m] = t.clamp(v, max=k - 1).to(t.int32)
        return out

    def lognormal_f32(self, mu, sigma, n):
        t = self.torch
        out = t.empty(n, dtype=t.float32, device=self.dev)
        step = 1 << 26
        for i in range(0, n, step):
            m = min(step, n - i)
            z = t.randn(m, generator=self.g, device=self.dev, dtype=t.float64)
            out[i:i + m] = t.exp(mu + sigma * z).to(t.float32)
        return out

    def add(self, a, b):
        return a + b

    def scale(self, a, m):
        return a * m


def _backend(seed, device):
    if device is None or device == "numpy":
        return _NumpyBackend(seed)
    return _TorchBackend(seed, device)


_ZIPF_CACHE = {}


def _zipf_cdf(s, k):
    """CDF of the bounded Zipf law P(v) ~ (v+1)^-s on v in [0, k), float64."""
    key = (s, k)
    if key not in _ZIPF_CACHE:
        w = np.arange(1, k + 1, dtype=np.float64) ** (-s)
        c = np.cumsum(w)
        _ZIPF_CACHE[key] = c / c[-1]
    return _ZIPF_CACHE[key]


def zipf_pmf0(s, k):
    """P(v = 0) of the bounded Zipf law, for tests of the generator."""
    w = np.arange(1, k + 1, dtype=np.float64) ** (-s)
    return 1.0 / w.sum()


# ---------------------------------------------------------------- tables

def table_plain(n=1_000_000, seed=None, device=None) -> Table:
    """The selection example of Section 1 on R(A, B, C, D).

    A = random permutation of 0..n-1, B ~ U[0,1000), C ~ U[0,10^6),
    D ~ Zipf(1.1) over [0,10^4)."""
    seed = data_seed(0) if seed is None else seed
    b = _backend(seed, device)
    cols = [b.perm(n), b.uniform(0, 1000, n), b.uniform(0, 1_000_000, n), b.zipf(1.1, 10_000, n)]
    return Table("R", n, [INT32] * 4, cols, ["perm", "uniform", "uniform", "zipf"],
                 [(0, n - 1), (0, 999), (0, 999_999), (0, 9_999)])


STAR_COLS = ["orderdate", "commitdate", "quantity", "discount", "price", "qty_key", "fk1", "fk2"]


def table_star(n=60_000_000, seed=None, device=None) -> Table:
    """Star-schema style fact table, 8 columns of 4 bytes.

    two date32 keys ~ U over 2,557 days from 1992-01-01; quantity U[1,50];
    discount U[0,10]; float32 price = exp(8 + N(0,1)); qty_key =
    10*quantity + U[0,10) (correlated with quantity); fk1, fk2 ~ Zipf(1.2)
    over 2*10^6 and 2*10^5 ids."""
    seed = data_seed(1) if seed is None else seed
    b = _backend(seed, device)
    od = b.uniform(DATE_LO, DATE_LO + DATE_SPAN, n)
    cd = b.uniform(DATE_LO, DATE_LO + DATE_SPAN, n)
    qty = b.uniform(1, 51, n)
    disc = b.uniform(0, 11, n)
    price = b.lognormal_f32(8.0, 1.0, n)
    qkey = b.add(b.scale(qty, 10), b.uniform(0, 10, n))
    fk1 = b.zipf(1.2, 2_000_000, n)
    fk2 = b.zipf(1.2, 200_000, n)
    return Table("lineorder", n, [DATE32, DATE32, INT32, INT32, FLOAT32, INT32, INT32, INT32],
                 [od, cd, qty, disc, price, qkey, fk1, fk2],
                 ["date", "date", "uniform", "uniform", "lognormal", "correlated", "zipf", "zipf"],
                 [(DATE_LO, DATE_LO + DATE_SPAN - 1)] * 2 + [(1, 50), (0, 10), None, (10, 509),
                                                            (0, 1_999_999), (0, 199_999)])


def table_mixed(n, ncols, seed, device=None, kinds=None) -> Table:
    """A table of the batched and learned workloads: column 0 a permutation
    key, the others drawn from uniform [0,10^4), Zipf(1.1) over [0,10^5),
    correlated (10 * an earlier uniform column + U[0,10)), uniform [0,10^6)
    and float32 lognormal."""
    b = _backend(seed, device)
    pick = np.random.default_rng(seed ^ 0x5EED)
    if kinds is None:
        pool = ["uniform", "zipf", "correlated", "uniform6", "lognormal"]
        kinds = ["perm"] + [pool[int(pick.integers(0, len(pool)))] for _ in range(ncols - 1)]
        if "correlated" in kinds:
            # a correlated column derives from an earlier uniform column
            first_c = kinds.index("correlated")
            if "uniform" not in kinds:
                kinds[first_c] = "uniform"
            elif kinds.index("uniform") > first_c:
                u = kinds.index("uniform")
                kinds[first_c], kinds[u] = "uniform", "correlated"
    cols, dtypes, domain = [], [], []
    for j, kd in enumerate(kinds):
        if kd == "perm":
            cols.append(b.perm(n)); dtypes.append(INT32); domain.append((0, max(n - 1, 0)))
        elif kd == "uniform":
            cols.append(b.uniform(0, 10_000, n)); dtypes.append(INT32); domain.append((0, 9_999))
        elif kd == "uniform6":
            cols.append(b.uniform(0, 1_000_000, n)); dtypes.append(INT32); domain.append((0, 999_999))
        elif kd == "zipf":
            cols.append(b.zipf(1.1, 100_000, n)); dtypes.append(INT32); domain.append((0, 99_999))
        elif kd == "correlated":
            src = kinds.index("uniform")
            cols.append(b.add(b.scale(cols[src], 10), b.uniform(0, 10, n)))
            dtypes.append(INT32); domain.append((0, 99_999))
        elif kd == "lognormal":
            cols.append(b.lognormal_f32(8.0, 1.0, n)); dtypes.append(FLOAT32); domain.append(None)
        else:
            raise ValueError(kd)
    return Table(f"t{n}", n, dtypes, cols, list(kinds), domain)


BATCH_SIZES = [10_000, 100_000, 1_000_000, 5_000_000, 20_000_000, 50_000_000, 100_000_000, 200_000_000]


def tables_batched(sizes=None, seed_base=None, device=None):
    """Eight tables of uneven sizes, 4..8 columns each."""
    sizes = BATCH_SIZES if sizes is None else sizes
    pick = np.random.default_rng(data_seed(2, 99))
    out = []
    for t, n in enumerate(sizes):
        ncols = int(pick.integers(4, 9))
        seed = data_seed(2, t) if seed_base is None else seed_base + t
        out.append(table_mixed(n, ncols, seed, device))
    return out


LEARNED_KINDS = ["perm", "uniform", "zipf", "correlated", "uniform6", "lognormal"]


def table_learned(n=100_000_000, seed=None, device=None) -> Table:
    """100M x 6 correlated / skewed table of the learned-gate workload."""
    seed = data_seed(3) if seed is None else seed
    return table_mixed(n, 6, seed, device, kinds=list(LEARNED_KINDS))


PLANNING_KINDS = ["perm", "uniform", "zipf", "correlated"]
PLANNING_SIZES = [10_000_000, 100_000_000, 1_000_000_000]


def tables_planning(sizes=None, device=None):
    """Three 4-column int32 tables of the planning workload."""
    sizes = PLANNING_SIZES if sizes is None else sizes
    return [table_mixed(n, 4, data_seed(4, t), device, kinds=list(PLANNING_KINDS))
            for t, n in enumerate(sizes)]


JOIN_SIZES = (10_000_000, 100_000_000, 1_000_000_000)


def tables_join(sizes=JOIN_SIZES, device=None):
    """Star schema of the join workload: build relations R and S (a key that
    is a permutation of 0..n-1 and an attribute: U[0,100) for R, bounded
    Zipf(1.1) over [0,10^5) for S) and the probe relation P with one foreign
    key into each, uniform over the referenced keys."""
    nr, ns, np_ = sizes
    br, bs, bp = _backend(data_seed(6, 0), device), _backend(data_seed(6, 1), device), _backend(data_seed(6, 2), device)
    R = Table("R", nr, [INT32, INT32], [br.perm(nr), br.uniform(0, 100, nr)], ["perm", "uniform"],
              [(0, nr - 1), (0, 99)])
    S = Table("S", ns, [INT32, INT32], [bs.perm(ns), bs.zipf(1.1, 100_000, ns)], ["perm", "zipf"],
              [(0, ns - 1), (0, 99_999)])
    P = Table("P", np_, [INT32, INT32], [bp.uniform(0, nr, np_), bp.uniform(0, ns, np_)], ["fk", "fk"],
              [(0, nr - 1), (0, ns - 1)])
    return R, S, P


# ---------------------------------------------------------------- TEXT and DECIMAL columns

def typed_vocab(k, seed):
    """k distinct strings: lowercase words of 1..12 letters drawn from a
    few shared stems (so that prefixes group many of them), a few with
    non-ASCII letters, and the empty string."""
    rng = np.random.default_rng(seed)
    stems = ["", "al", "bra", "ca", "car", "dark", "gold", "ivo", "lin", "ma", "mi", "ro", "sa", "sm"]
    extra = ["é", "ü", "ß", "中", "~"]
    letters = np.array(list("abcdefghijklmnopqrstuvwxyz"))
    out = {""}
    while len(out) < k:
        w = stems[rng.integers(len(stems))] + "".join(rng.choice(letters, rng.integers(0, 9)))
        if rng.random() < 0.03:
            w += extra[rng.integers(len(extra))]
        out.add(w[:12])
    return sorted(out, key=lambda x: rng.random())   # no particular order


def typed_columns(n, seed):
    """Columns of the TEXT / DECIMAL workload (Section 3, Table 3): a TEXT
    column given as indices into `vocab` (bounded Zipf(1.05) over 2,000
    strings), a DECIMAL(15,2) price as hundredths in [90,000, 10,500,000)
    (900.00 .. 104,999.99), a DECIMAL(15,2) discount in hundredths 0..10
    (0.00 .. 0.10) and an INTEGER quantity 1..50."""
    rng = np.random.default_rng(seed)
    vocab = typed_vocab(2000, seed + 1)
    cdf = _zipf_cdf(1.05, len(vocab))
    idx = np.minimum(np.searchsorted(cdf, rng.random(n), side="right"), len(vocab) - 1).astype(np.int32)
    price = rng.integers(90_000, 10_500_000, n).astype(np.int32)
    disc = rng.integers(0, 11, n).astype(np.int32)
    qty = rng.integers(1, 51, n).astype(np.int32)
    return vocab, idx, price, disc, qty


WIDE_EDGES = [0, -1, 1, 2**31 - 1, 2**31, 2**32 - 1, 2**32, 2**32 + 1, -2**31, -2**31 - 1, -2**32,
              -2**32 - 1, 10**15 - 1, -(10**15 - 1)]


def typed_wide(n, seed):
    """A DECIMAL(15,2) column beyond the int32 range, as int64 hundredths:
    magnitude 10^U(0,15) (log-uniform over the whole precision), negative
    with probability 0.2, and 1 % of the rows at the 32-bit word edges
    (+-2^31, +-2^32, ...) and at +-(10^15 - 1)."""
    rng = np.random.default_rng(seed)
    mag = np.minimum(np.floor(10.0 ** rng.uniform(0, 15, n)), 10**15 - 1).astype(np.int64)
    x = np.where(rng.random(n) < 0.2, -mag, mag)
    edge = rng.random(n) < 0.01
    x[edge] = np.array(WIDE_EDGES, dtype=np.int64)[rng.integers(0, len(WIDE_EDGES), int(edge.sum()))]
    return x


def _wide_literal(rng, present):
    r = rng.random()
    if r < 0.3 and len(present):
        v = int(present[rng.integers(len(present))])          # a stored value, exactly
        return ("-" if v < 0 else "") + "%d.%02d" % divmod(abs(v), 100)
    if r < 0.45:
        v = WIDE_EDGES[rng.integers(len(WIDE_EDGES))] + int(rng.integers(-1, 2))
        return ("-" if v < 0 else "") + "%d.%02d" % divmod(abs(v), 100)
    d = int(rng.integers(0, 5))
    v = 10.0 ** rng.uniform(-2, 13.2) * (-1 if rng.random() < 0.3 else 1)
    return ("%.*f" % (d, v)) if d else str(int(v))


def _dec_literal(rng, lo, hi):
    """A decimal literal between lo and hi (in units) with 0..4 decimals."""
    d = int(rng.integers(0, 5))
    v = rng.uniform(lo, hi)
    return ("%.*f" % (d, v)) if d else str(int(round(v)))


def typed_preds(vocab, rng, count, wide=None):
    """Predicates over (text, price, discount, quantity) = columns 0..3 in
    the typed leaf forms: strings on column 0 (present ones, absent ones,
    prefixes), decimal literals on columns 1 and 2 (some with more decimals
    than the scale, some outside the stored range) and ints on column 3.
    With `wide` (a sample of a typed_wide column's values), column 4 is
    that DECIMAL(15,2) column, with literals from its values, its word
    edges and log-uniform magnitudes."""
    def s_any():
        r = rng.random()
        w = vocab[rng.integers(len(vocab))]
        if r < 0.6:
            return w
        if r < 0.8:
            return w + "m"             # most likely absent
        return w[: int(rng.integers(0, len(w) + 1))]

    def leaf():
        c = int(rng.integers(0, 5 if wide is not None else 4))
        if c == 4:
            op = ["eq", "lt", "gt", "between", "in"][rng.integers(5)]
            if op == "between":
                a, b = _wide_literal(rng, wide), _wide_literal(rng, wide)
                if rng.random() < 0.8 and float(a) > float(b):
                    a, b = b, a
                return ("between", 4, a, b)
            if op == "in":
                return ("in", 4, [_wide_literal(rng, wide) for _ in range(int(rng.integers(1, 6)))])
            return (op, 4, _wide_literal(rng, wide))
        if c == 0:
            op = ["eq", "lt", "gt", "between", "in", "prefix"][rng.integers(6)]
            if op == "between":
                a, b = sorted([s_any(), s_any()])
                return ("between", 0, a, b) if rng.random() < 0.9 else ("between", 0, b, a)
            if op == "in":
                return ("in", 0, [s_any() for _ in range(int(rng.integers(1, 6)))])
            if op == "prefix":
                w = vocab[rng.integers(len(vocab))]
                return ("prefix", 0, w[: int(rng.integers(0, 4))])
            return (op, 0, s_any())
        if c in (1, 2):
            lo, hi = (900.0, 105_000.0) if c == 1 else (-0.02, 0.12)
            if rng.random() < 0.05:
                lo, hi = (-1e12, 1e12)     # far outside int32 hundredths
            op = ["eq", "lt", "gt", "between", "in"][rng.integers(5)]
            if op == "between":
                a, b = _dec_literal(rng, lo, hi), _dec_literal(rng, lo, hi)
                return ("between", c, a, b)
            if op == "in":
                return ("in", c, [_dec_literal(rng, lo, hi) for _ in range(int(rng.integers(1, 5)))])
            if op == "eq" and c == 2:
                return ("eq", 2, "0.0%d" % rng.integers(0, 10))
            return (op, c, _dec_literal(rng, lo, hi))
        op = ["eq", "lt", "gt", "between"][rng.integers(4)]
        if op == "between":
            a = int(rng.integers(0, 52))
            return ("between", 3, a, a + int(rng.integers(0, 20)))
        return (op, 3, int(rng.integers(0, 52)))

    out = []
    for _ in range(count):
        k = int(rng.integers(1, 4))
        if k == 1:
            out.append(leaf())
        elif rng.random() < 0.7:
            out.append(("and", [leaf() for _ in range(k)]))
        else:
            out.append(("and", [leaf(), ("or", [leaf() for _ in range(k)])]))
    return out


# ---------------------------------------------------------------- special tables for pins

def table_edge_floats() -> Table:
    """Hand-built float32 column with NaN, +-0, +-inf, denormals and normals,
    next to an int32 column with the int32 extremes."""
    f = np.array([np.nan, -np.nan, 0.0, -0.0, np.inf, -np.inf,
                  1e-45, -1e-45, 1.1754942e-38, 1.17549435e-38, -1.17549435e-38,
                  1.0, -1.0, 2.5, 3.4028235e38, -3.4028235e38], dtype=np.float32)
    i = np.array([-2**31, 2**31 - 1, 0, -1, 1, 7, -7, 2**30,
                  -2**30, 100, -100, 5, 5, 5, 2**31 - 2, -2**31 + 1], dtype=np.int32)
    return Table("edges", len(f), [FLOAT32, INT32], [f, i], ["edge", "edge"], [None, (-2**31, 2**31 - 1)])


# ---------------------------------------------------------------- value helpers

def _val(col, i):
    v = col[int(i)]
    if hasattr(v, "item"):
        v = v.item()
    return v


def _row_values(col, idx):
    if isinstance(col, np.ndarray):
        return col[idx]
    import torch
    return col[torch.as_tensor(idx, device=col.device, dtype=torch.int64)].cpu().numpy()


def _const(dtype, v):
    return np.float32(v) if dtype == FLOAT32 else int(v)


# ---------------------------------------------------------------- predicates

UDF_PLAIN = ("mod", ("add", ("mul", ("col", 1), ("const", 31)), ("col", 3)), ("const", 97))


def pred_plain(table: Table, seed: int):
    """Constants of the Section 1 selection drawn from the seed, in the order
    x, (y1, y2), z1, z2, w:

        B = x AND C BETWEEN y1, y2 AND (D = z1 OR D > z2) AND (31*B + D) mod 97 > w
    """
    rng = np.random.default_rng(seed)
    x = int(rng.integers(0, 1000))
    y = sorted(int(v) for v in rng.integers(0, 1_000_000, 2))
    z1 = int(_row_values(table.cols[3], np.array([int(rng.integers(0, table.nrows))]))[0]) if table.nrows else 0
    z2 = int(rng.integers(0, 10_000))
    w = int(rng.integers(0, 97))
    return ("and", [("eq", 1, x), ("between", 2, y[0], y[1]),
                    ("or", [("eq", 3, z1), ("gt", 3, z2)]),
                    ("udf", UDF_PLAIN, ("gt", w))])


PLAIN_PROJECTION = [0, 2, 3]   # A, C, D: the pushed-down projection of Section 2
STAR_PROJECTION = [6, 7, 4]    # fk1, fk2, price


def _rows(table, rng, m):
    return rng.integers(0, max(table.nrows, 1), m)


def _leaf_star(table, c, rng, force=None):
    kind = table.kinds[c]
    col = table.cols[c]
    if kind == "date":
        op = force or rng.choice(["between", "between", "between", "lt", "gt"])
        d = int(rng.integers(DATE_LO, DATE_LO + DATE_SPAN))
        if op == "between":
            w = int(rng.integers(1, 367))
            return ("between", c, d, d + w - 1)
        return (op, c, d)
    if c in (2, 3):
        lo, hi = table.domain[c]
        op = force or rng.choice(["eq", "between", "in"])
        if op == "eq":
            return ("eq", c, int(rng.integers(lo, hi + 1)))
        if op == "between":
            a, b = sorted(int(v) for v in rng.integers(lo, hi + 1, 2))
            return ("between", c, a, b)
        m = int(rng.integers(1, min(16, hi - lo + 1) + 1))
        return ("in", c, [int(v) for v in rng.integers(lo, hi + 1, m)])
    if kind == "lognormal":
        op = force or rng.choice(["lt", "gt", "between"])
        vals = _row_values(col, _rows(table, rng, 2)) if table.nrows else np.zeros(2, np.float32)
        if op == "between":
            a, b = sorted(vals.tolist())
            return ("between", c, np.float32(a), np.float32(b))
        return (op, c, np.float32(vals[0]))
    if kind == "correlated":
        lo, hi = table.domain[c]
        op = force or rng.choice(["between", "lt", "gt"])
        if op == "between":
            a = int(rng.integers(lo, hi + 1))
            return ("between", c, a, a + int(rng.integers(0, 60)))
        return (op, c, int(rng.integers(lo, hi + 1)))
    # zipf foreign keys: = or IN of 1..16 values drawn from rows, so they hit
    op = force or rng.choice(["eq", "in"])
    if op == "eq":
        v = _row_values(col, _rows(table, rng, 1)) if table.nrows else np.zeros(1, np.int32)
        return ("eq", c, int(v[0]))
    m = int(rng.integers(1, 17))
    v = _row_values(col, _rows(table, rng, m)) if table.nrows else np.zeros(m, np.int32)
    return ("in", c, [int(x) for x in v])


def preds_star(table: Table, count=32, seed=None):
    """Random conjunctions of 2..5 leaves on distinct columns of the star
    table.  The first four cover a date range, a BETWEEN on an int column,
    an IN-list and a float comparison."""
    rng = np.random.default_rng(pred_seed(1) if seed is None else seed)
    forced = [(0, "between"), (2, "between"), (6, "in"), (4, "lt")]
    out = []
    for p in range(count):
        k = int(rng.integers(2, 6))
        cols = [int(c) for c in rng.choice(8, k, replace=False)]
        fc, force = forced[p] if p < len(forced) else (-1, None)
        if fc >= 0 and fc not in cols:
            cols[0] = fc
        leaves = [_leaf_star(table, c, rng, force if c == fc else None) for c in cols]
        out.append(("and", leaves))
    return out


def _leaf_mixed(table, c, rng):
    kind = table.kinds[c]
    col = table.cols[c]
    n = table.nrows
    if kind == "lognormal":
        op = rng.choice(["lt", "gt", "between"])
        vals = _row_values(col, _rows(table, rng, 2)) if n else np.zeros(2, np.float32)
        if op == "between":
            a, b = sorted(vals.tolist())
            return ("between", c, np.float32(a), np.float32(b))
        return (str(op), c, np.float32(vals[0]))
    lo, hi = table.domain[c]
    span = hi - lo + 1
    if kind == "zipf":
        op = rng.choice(["eq", "in", "lt", "gt"])
    elif kind == "perm":
        op = rng.choice(["lt", "gt", "between", "eq"])
    else:
        op = rng.choice(["eq", "lt", "gt", "between", "between", "in"])
    if op in ("eq", "in") and kind in ("zipf", "correlated"):
        m = 1 if op == "eq" else int(rng.integers(2, 17))
        v = _row_values(col, _rows(table, rng, m)) if n else np.zeros(m, np.int32)
        return ("eq", c, int(v[0])) if op == "eq" else ("in", c, [int(x) for x in v])
    if op == "eq":
        return ("eq", c, int(rng.integers(lo, hi + 1)))
    if op == "in":
        m = int(rng.integers(2, 17))
        return ("in", c, [int(x) for x in rng.integers(lo, hi + 1, m)])
    # ranges with log-uniform width so that selectivities spread over decades
    frac = 10.0 ** rng.uniform(-5, 0)
    width = max(1, int(frac * span))
    if op == "between":
        a = int(rng.integers(lo, max(lo + 1, hi - width + 2)))
        return ("between", c, a, min(hi, a + width - 1))
    if op == "lt":
        return ("lt", c, lo + width)
    return ("gt", c, hi - width)


def preds_mixed(table: Table, count, seed, min_conj=1, max_conj=6, p_or=0.3):
    """Conjunctions of min_conj..max_conj conjuncts; columns may repeat; a
    conjunct is a single leaf (probability 1 - p_or) or an OR of two leaves."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        k = int(rng.integers(min_conj, max_conj + 1))
        conj = []
        for _ in range(k):
            if rng.random() < p_or:
                a, b = (int(c) for c in rng.integers(0, len(table.cols), 2))
                conj.append(("or", [_leaf_mixed(table, a, rng), _leaf_mixed(table, b, rng)]))
            else:
                conj.append(_leaf_mixed(table, int(rng.integers(0, len(table.cols))), rng))
        out.append(("and", conj) if len(conj) > 1 else conj[0])
    return out


def _leaf_around(table, c, v, rng):
    """A leaf on column c that row value v satisfies; widths log-uniform so
    that selectivities spread over decades."""
    kind = table.kinds[c]
    frac = 10.0 ** rng.uniform(-5, 0)
    if kind == "lognormal":
        v = np.float32(v)
        op = rng.choice(["lt", "gt", "between"])
        up = np.float32(v * (1.0 + frac * 20.0) + 1e-3)
        dn = np.float32(max(0.0, v * (1.0 - frac) - 1e-3))
        up = up if up > v else np.nextafter(v, np.float32(np.inf))
        dn = dn if dn < v else np.nextafter(v, np.float32(-np.inf))
        if op == "lt":
            return ("lt", c, up)
        if op == "gt":
            return ("gt", c, dn)
        return ("between", c, dn, up)
    v = int(v)
    lo, hi = table.domain[c]
    w = max(1, int(frac * (hi - lo + 1)))
    op = rng.choice(["eq", "lt", "gt", "between", "between", "in"] if kind != "perm" else ["lt", "gt", "between"])
    if op == "eq":
        return ("eq", c, v)
    if op == "lt":
        return ("lt", c, v + 1 + int(rng.integers(0, w)))
    if op == "gt":
        return ("gt", c, v - 1 - int(rng.integers(0, w)))
    if op == "between":
        a = int(rng.integers(0, w))
        return ("between", c, v - a, v + (w - a))
    m = int(rng.integers(2, 17))
    vals = [v] + [int(x) for x in rng.integers(lo, hi + 1, m - 1)]
    rng.shuffle(vals)
    return ("in", c, vals)


def preds_anchored(table: Table, count, seed, min_conj=1, max_conj=4, p_or=0.2):
    """Conjunctions built around a sampled row: every conjunct holds for
    that row (an OR pairs a leaf it satisfies with a random leaf), so each
    predicate selects at least one row; conjuncts are on distinct columns."""
    rng = np.random.default_rng(seed)
    n, ncols = table.nrows, len(table.cols)
    rows = rng.integers(0, max(n, 1), count)
    vals = [np.asarray(_row_values(col, rows)) for col in table.cols]
    out = []
    for i in range(count):
        k = int(rng.integers(min_conj, min(max_conj, ncols) + 1))
        cols = [int(c) for c in rng.choice(ncols, k, replace=False)]
        conj = []
        for c in cols:
            leaf = _leaf_around(table, c, vals[c][i], rng)
            if rng.random() < p_or:
                other = int(rng.integers(0, ncols))
                leaf = ("or", [leaf, _leaf_mixed(table, other, rng)])
            conj.append(leaf)
        out.append(("and", conj) if len(conj) > 1 else conj[0])
    return out


def preds_batched(tables, per_table=32, seed=None):
    """32 predicates per table (256 over the eight tables); returns
    (predicates, table index of each)."""
    seed = pred_seed(2) if seed is None else seed
    preds, owner = [], []
    for t, tab in enumerate(tables):
        ps = preds_mixed(tab, per_table, seed + t)
        preds += ps
        owner += [t] * len(ps)
    return preds, owner


def random_pred_tiny(table: Table, rng, depth=0, udf=True):
    """Arbitrary AND/OR trees over every leaf kind, for brute-force checks on
    tiny tables (constants drawn from the column's values and their
    neighbours, so boundaries are hit)."""
    ncols = len(table.cols)
    r = rng.random()
    if depth < 3 and r < 0.35:
        kids = [random_pred_tiny(table, rng, depth + 1, udf) for _ in range(int(rng.integers(1, 4)))]
        return ("and" if rng.random() < 0.5 else "or", kids)
    int_cols = [c for c in range(ncols) if table.dtypes[c] != FLOAT32]
    if udf and int_cols and rng.random() < 0.15:
        expr = ("col", int(rng.choice(int_cols)))
        for _ in range(int(rng.integers(1, 4))):
            op = str(rng.choice(["add", "sub", "mul", "mod", "band", "bor", "bxor", "shl", "shr"]))
            if op == "mod":
                rhs = ("const", int(rng.integers(1, 50)))
            elif op in ("shl", "shr"):
                rhs = ("const", int(rng.integers(0, 32)))
            elif rng.random() < 0.5:
                rhs = ("col", int(rng.choice(int_cols)))
            else:
                rhs = ("const", int(rng.integers(-100, 100)))
            expr = (op, expr, rhs)
        k = [int(v) for v in rng.integers(-50, 50, 3)]
        tk = str(rng.choice(["eq", "lt", "gt", "between", "in"]))
        test = {"eq": ("eq", k[0]), "lt": ("lt", k[0]), "gt": ("gt", k[0]),
                "between": ("between", min(k[0], k[1]), max(k[0], k[1])), "in": ("in", k)}[tk]
        return ("udf", expr, test)
    c = int(rng.integers(0, ncols))
    col = table.cols[c]
    dt = table.dtypes[c]

    def pick():
        if table.nrows and rng.random() < 0.8:
            v = _val(col, rng.integers(0, table.nrows))
            if dt != FLOAT32:
                v = int(v) + int(rng.integers(-1, 2))
                v = max(-2**31, min(2**31 - 1, v))
            return _const(dt, v)
        if dt == FLOAT32:
            return np.float32(rng.choice([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, 1.0, -1.0]))
        return int(rng.choice([-2**31, 2**31 - 1, 0, -1, 1]))

    op = str(rng.choice(["eq", "lt", "gt", "between", "in"]))
    if op == "between":
        a, b = pick(), pick()
        if rng.random() < 0.8 and not (dt == FLOAT32 and (np.isnan(a) or np.isnan(b))):
            a, b = (a, b) if a <= b else (b, a)
        return ("between", c, a, b)
    if op == "in":
        return ("in", c, [pick() for _ in range(int(rng.integers(1, 6)))])
    return (op, c, pick())


# ---------------------------------------------------------------- MLP inputs

MLP_DIMS = (64, 256, 256, 256, 1)


def mlp_init(seed=MLP_SEED, dims=MLP_DIMS):
    """He-uniform weights (U(-sqrt(6/fan_in), +sqrt(6/fan_in))) and zero
    biases, float32, weights stored [fan_in, fan_out]."""
    rng = np.random.default_rng(seed)
    params = []
    for i in range(len(dims) - 1):
        a = math.sqrt(6.0 / dims[i])
        w = rng.uniform(-a, a, (dims[i], dims[i + 1])).astype(np.float32)
        params.append((w, np.zeros(dims[i + 1], np.float32)))
    return params


def minibatch_order(n, batch, epochs, seed):
    """Sample order for minibatch training: one seeded permutation of
    [0, n) per epoch, truncated to whole batches, int32."""
    rng = np.random.default_rng(seed)
    steps = n // batch
    out = [rng.permutation(n)[: steps * batch] for _ in range(epochs)]
    return np.concatenate(out).astype(np.int32) if out else np.zeros(0, np.int32)


def poisson_arrivals(nq, rate_per_s, seed):
    """Arrival times (seconds) of a seeded Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, nq))
