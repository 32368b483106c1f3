"""Pins of the MLP, featurization and gate oracles.

- backward vs central finite differences of the float64 network (catches a
  transposed operand, a missing ReLU mask, a wrong sign or scale);
- forward on a hand-built network whose output is known in closed form;
- bfloat16 rounding against hand-picked bit patterns (ties to even);
- Adam's first steps in closed form;
- featurization of hand-worked predicates (tests/golden/features.txt);
- gate decisions at hand-computed points.
"""
import math
import os

import numpy as np
import pytest

from oracle import features as fo
from oracle import mlp
from paper_1901_01488_amd import datagen as dg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny_params(rng, dims=(5, 7, 6, 4, 1)):
    return [(rng.normal(0, 0.7, (dims[i], dims[i + 1])), rng.normal(0, 0.3, dims[i + 1]))
            for i in range(len(dims) - 1)]


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = _tiny_params(rng)
    x = rng.normal(0, 1, (9, 5))
    y = rng.normal(0, 1, 9)

    def L(p):
        yh, _ = mlp.forward(p, x, rounding=False)
        return mlp.loss(yh, y)

    yh, acts = mlp.forward(params, x, rounding=False)
    grads = mlp.backward(params, acts, yh, y, rounding=False)
    h = 1e-6
    for li, (w, b) in enumerate(params):
        for which, arr in ((0, w), (1, b)):
            g = np.asarray(grads[li][which]).reshape(arr.shape)
            for idx in np.ndindex(arr.shape):
                def bump(s):
                    q = [[np.array(a, np.float64, copy=True) for a in layer] for layer in params]
                    q[li][which][idx] += s
                    return [tuple(layer) for layer in q]
                fd = (L(bump(h)) - L(bump(-h))) / (2 * h)
                assert abs(fd - g[idx]) <= 1e-6 + 1e-4 * abs(fd), (li, which, idx, fd, g[idx])


def test_forward_closed_form():
    # layer 1 copies the positive part of each input (x and -x lanes), the
    # next layers pass through, the head sums: y = sum |x_i| + 0.5
    d = 3
    w1 = np.concatenate([np.eye(d), -np.eye(d)], axis=1)
    w2 = np.eye(2 * d)
    w3 = np.eye(2 * d)
    w4 = np.ones((2 * d, 1))
    params = [(w1, np.zeros(2 * d)), (w2, np.zeros(2 * d)), (w3, np.zeros(2 * d)), (w4, np.array([0.5]))]
    x = np.array([[1.0, -2.0, 0.25], [0.0, 0.0, 0.0], [-3.0, 4.0, -0.5]])
    yh, _ = mlp.forward(params, x, rounding=False)
    assert np.allclose(yh, [3.75, 0.5, 8.0], atol=0, rtol=0)
    # bf16-exact inputs give the same numbers with rounding on
    yh2, _ = mlp.forward(params, x, rounding=True)
    assert np.array_equal(yh2, yh)


def test_bf16_rounding_bits():
    cases = {
        0x3F800000: 0x3F800000,   # 1.0 exact
        0x3F808000: 0x3F800000,   # tie, even mantissa stays
        0x3F818000: 0x3F820000,   # tie, odd mantissa rounds up
        0x3F808001: 0x3F810000,   # above the tie
        0x3F807FFF: 0x3F800000,   # below the tie
        0xBF818000: 0xBF820000,   # negative tie to even
        0x7F7FFFFF: 0x7F800000,   # largest float rounds to +inf
        0x00000001: 0x00000000,   # smallest denormal rounds to 0
    }
    for src, want in cases.items():
        x = np.array([src], np.uint32).view(np.float32)
        got = np.float32(mlp.bf16(x)[0]).view(np.uint32)
        assert int(got) == want, hex(src)
    assert np.isnan(mlp.bf16(np.array([np.nan], np.float32))[0])


def test_adam_first_steps_closed_form():
    w = np.array([[0.5, -0.25]], np.float32)
    b = np.array([1.0], np.float32)
    opt = mlp.Adam([(w, b)], lr=0.01)
    g = [(np.array([[2.0, -0.5]]), np.array([0.0]))]
    (w1, b1), = opt.step([(w, b)], g)
    # step 1: m_hat = g, v_hat = g^2, update = lr * g / (|g| + eps)
    assert np.allclose(w1, w - 0.01 * np.sign([[2.0, -0.5]]), rtol=0, atol=1e-7)
    assert b1[0] == b[0]
    (w2, _), = opt.step([(w1, b1)], g)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    assert np.allclose(w2, w1 - 0.01 * np.sign([[2.0, -0.5]]), rtol=0, atol=1e-7)
    # a gradient that flips sign at step 2: m = 0.09 g - 0.1 g... worked out by hand
    opt2 = mlp.Adam([(w, b)], lr=1.0)
    gg = np.array([[1.0, 1.0]])
    opt2.step([(w, b)], [(gg, np.zeros(1))])
    (w3, _), = opt2.step([(w, b)], [(-gg, np.zeros(1))])
    m = 0.9 * 0.1 * 1 + 0.1 * (-1)        # -0.01
    v = 0.999 * 0.001 * 1 + 0.001 * 1     # 0.001999
    upd = (m / (1 - 0.81)) / (math.sqrt(v / (1 - 0.998001)) + 1e-8)
    assert np.allclose(w3, w - upd, rtol=1e-6, atol=0)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    x = rng.normal(0, 1, (256, 64)).astype(np.float32)
    y = (x[:, 0] * 2 - x[:, 1]).astype(np.float32)
    params = dg.mlp_init(7)
    order = dg.minibatch_order(256, 64, 6, seed=4)
    _, losses = mlp.train(params, x, y, order, 64, lr=1e-3)
    assert np.mean(losses[-4:]) < 0.5 * np.mean(losses[:4])


def test_q_error_and_label():
    assert mlp.q_error(10, 10, 100)[()] == 1.0
    assert mlp.q_error(20, 10, 100)[()] == 2.0
    assert mlp.q_error(0.001, 0, 100)[()] == 1.0      # both clamp to 1
    assert mlp.q_error(1e9, 50, 100)[()] == 2.0       # c_hat clamps to n
    assert mlp.label(0, 1000)[()] == math.log(1 / 1000)
    assert mlp.label(1000, 1000)[()] == 0.0


# ----------------------------------------------------------- featurization

GOLDEN_MIN = [0, 0, 0, 0, 0, np.float32(1.0)]
GOLDEN_MAX = [100, 9, 1000, 1, 0, np.float32(3.0)]
GOLDEN_DTYPES = "iiiiif"


def _read_feature_golden():
    """Cases of tests/golden/features.txt: {"pred", "sample", "nz"}."""
    cases = []
    sample = None
    with open(os.path.join(GOLDEN, "features.txt")) as f:
        cur = None
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line == "sample none":
                sample = None
            elif line.startswith("sample "):
                c, vals = line[7:].split(":")
                sample = dict(sample or {})
                sample[int(c)] = [float(v) if GOLDEN_DTYPES[int(c)] == "f" else int(v) for v in vals.split()]
            elif line.startswith("pred "):
                cur = {"pred": eval(line[5:], {"np": np}), "nz": {}, "sample": sample}   # fixture literal, written by hand
                cases.append(cur)
            else:
                k, v = line.split("=")
                cur["nz"][int(k)] = float(v)
    return cases


def golden_sample(case):
    s = case["sample"]
    return None if s is None else [s[c] for c in range(6)]


def test_featurize_golden():
    for case in _read_feature_golden():
        cat = fo.Catalog(GOLDEN_MIN, GOLDEN_MAX, GOLDEN_DTYPES, golden_sample(case))
        f = fo.featurize(case["pred"], cat)
        want = np.zeros(64, np.float32)
        for c in range(6):
            want[10 * c + 2] = 1.0
        for k, v in case["nz"].items():
            want[k] = np.float32(v)
        assert np.array_equal(f, want), (case["pred"], np.flatnonzero(f != want), f[f != want])


def test_column_cdf_properties():
    """The smoothed CDF is monotone, 0 below the minimum and 1 above the
    maximum, and the mass of an integer column's cells sums to 1."""
    rng = np.random.default_rng(8)
    for _ in range(20):
        smp = rng.zipf(1.3, 300) % 50
        cdf = fo.ColumnCdf(0, 60, True, smp)
        cells = [cdf.atmost(k) - cdf.below(k) for k in range(0, 61)]
        assert all(c >= 0 for c in cells)
        assert abs(sum(cells) - 1.0) < 1e-12
        vals = [cdf.atmost(k) for k in range(-3, 64)]
        assert all(a <= b for a, b in zip(vals, vals[1:]))
        assert cdf.below(0) == 0.0 and cdf.atmost(60) == 1.0
        # a value sampled r times carries a jump of (r - 1) / m plus its cell
        v = int(np.bincount(smp).argmax())
        r = int((smp == v).sum())
        assert cdf.atmost(v) - cdf.below(v) >= (r - 1) / len(smp) - 1e-12
    f = fo.ColumnCdf(-1.0, 1.0, False, rng.standard_normal(500).clip(-1, 1))
    xs = np.linspace(-1.5, 1.5, 301)
    ys = [f.atmost(x) for x in xs]
    assert all(a <= b for a, b in zip(ys, ys[1:])) and ys[0] == 0.0 and ys[-1] == 1.0


# ----------------------------------------------------------- gate

def test_gate_pushdown_band():
    n = 10**8
    tau, beta = 0.05, 2.0
    # selectivity exactly tau: inside; tau*beta*1.01 outside; tau/beta/1.01 outside
    assert fo.route_pushdown(math.log(tau), n, tau, beta, 10**6)
    assert not fo.route_pushdown(math.log(tau * beta * 1.01), n, tau, beta, 10**6)
    assert not fo.route_pushdown(math.log(tau / beta / 1.01), n, tau, beta, 10**6)
    assert fo.route_pushdown(math.log(tau * beta * 0.99), n, tau, beta, 10**6)
    # small tables are never materialized, so never routed
    assert not fo.route_pushdown(math.log(tau), 10**5, tau, beta, 10**6)
    # predictions above 0 clamp to selectivity 1, below ln(1/n) to 1/n
    assert not fo.route_pushdown(5.0, n, tau, beta, 10**6)
    assert fo.route_pushdown(5.0, n, 0.9, 2.0, 10**6)


def test_gate_join_pair():
    beta = 1.5
    # c_R = 1000, c_S = 2000 -> ratio 0.5 < 1/beta^2 = 0.444? no: 0.5 >= 0.444 -> routed
    yr = math.log(1000 / 10**7)
    ys = math.log(2000 / 10**8)
    assert fo.route_join_pair(yr, 10**7, ys, 10**8, beta)
    ys2 = math.log(3000 / 10**8)     # ratio 1/3 < 0.444 -> order is safe
    assert not fo.route_join_pair(yr, 10**7, ys2, 10**8, beta)


def test_gate_join_tie():
    beta = 1.5
    # c_R = 1000 of 10^7 (sel 1e-4), c_S = 2000 of 10^8 (sel 2e-5): the
    # orders could flip (ratio 0.5 >= 1/beta^2), but at the top of the band
    # the selectivities are 1.5e-4 and 3e-5, both below tie_sel = 1e-3
    yr = math.log(1000 / 10**7)
    ys = math.log(2000 / 10**8)
    assert fo.route_join_pair(yr, 10**7, ys, 10**8, beta, tie_sel=0.0)
    assert not fo.route_join_pair(yr, 10**7, ys, 10**8, beta, tie_sel=1e-3)
    # tie_sel = 1e-4: R's band reaches 1.5e-4 > 1e-4, so the pair is routed
    assert fo.route_join_pair(yr, 10**7, ys, 10**8, beta, tie_sel=1e-4)
    # boundary: R's selectivity times beta exactly tie_sel is a tie
    yr_edge = math.log(1e-3 / beta)
    ys_edge = math.log(1e-3 / beta) + math.log(10**7 / 10**8)   # same filtered size as R
    assert not fo.route_join_pair(yr_edge, 10**7, ys_edge, 10**8, beta, tie_sel=1e-3 * (1 + 1e-12))
    assert fo.route_join_pair(yr_edge, 10**7, ys_edge, 10**8, beta, tie_sel=1e-3 * (1 - 1e-9))
    # two empty selections (estimates clamped to one row each): equal
    # filtered sizes route without ties, and are a tie once tie_sel >= beta / n
    assert fo.route_join_pair(-50.0, 10**7, -50.0, 10**8, beta)
    assert not fo.route_join_pair(-50.0, 10**7, -50.0, 10**7, beta, tie_sel=1e-6)
    assert fo.route_join_pair(-50.0, 10**7, -50.0, 10**7, beta, tie_sel=0.0)


def test_huber_loss_values():
    # e^2 / 2 inside the threshold 1/2, 1/2 (|e| - 1/4) beyond; continuous at |e| = 1/2
    assert mlp.loss(np.array([0.25]), np.array([0.0])) == 0.03125
    assert mlp.loss(np.array([-2.0]), np.array([0.0])) == 0.875
    assert mlp.loss(np.array([0.5]), np.array([0.0])) == 0.125
    assert mlp.loss(np.array([3.0, 1.0]), np.array([3.0, 0.75])) == 0.015625
