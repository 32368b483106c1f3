"""GPU parity of the MLP estimator (bf16 MFMA forward / backward, Adam)
against the CPU oracle with the same rounding points."""
import numpy as np
import pytest

from oracle import mlp as om
from paper_1901_01488_amd import datagen as dg
from paper_1901_01488_amd import esc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    torch.cuda.init()
    return esc.Context(0)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def test_single_tile_layout(ctx):
    """One 32x32 output tile through a 64->256 layer with hand-made weights:
    checks the MFMA operand and accumulator lane layout exactly."""
    import torch
    params = dg.mlp_init(7)
    # layer 1 = a permutation-like sparse matrix of small integers, other layers identity-like
    w1 = np.zeros((64, 256), np.float32)
    for i in range(64):
        w1[i, (5 * i + 3) % 256] = float(i % 7 + 1)
        w1[i, (11 * i) % 256] += 2.0
    params[0] = (w1, np.arange(256, dtype=np.float32) * 0.0)
    x = np.zeros((37, 64), np.float32)
    for r in range(37):
        x[r, (r * 3) % 64] = float(r % 5 + 1)
        x[r, (r * 7 + 1) % 64] = -1.0
    m = esc.MLP(ctx, params)
    xt = torch.from_numpy(x).cuda()
    got = m.predict(xt).cpu().numpy()
    want, _ = om.forward(params, x)
    assert np.allclose(got, want, rtol=2e-2, atol=1e-3), (got[:5], want[:5])


@pytest.mark.parametrize("n", [1, 33, 100, 512, 4096, 5000])
def test_forward_matches_oracle(ctx, n):
    import torch
    rng = np.random.default_rng(n)
    x = rng.normal(0, 1, (n, 64)).astype(np.float32)
    params = dg.mlp_init(7)
    m = esc.MLP(ctx, params)
    got = m.predict(torch.from_numpy(x).cuda()).cpu().numpy()
    want, _ = om.forward(params, x)
    assert rel(got, want) < 1e-2
    assert np.max(np.abs(got - want)) < 2e-2 * max(1.0, np.max(np.abs(want)))


@pytest.mark.parametrize("n", [7, 256, 1024])
def test_gradients_match_oracle(ctx, n):
    import torch
    rng = np.random.default_rng(100 + n)
    x = rng.normal(0, 1, (n, 64)).astype(np.float32)
    y = rng.normal(-5, 2, n).astype(np.float32)
    params = dg.mlp_init(7)
    m = esc.MLP(ctx, params)
    g = m.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
    yh, acts = om.forward(params, x)
    want = om.backward(params, acts, yh, y)
    got = esc.flat_to_params(g)
    for li, ((gw, gb), (ww, wb)) in enumerate(zip(got, want)):
        assert rel(gw, np.asarray(ww).reshape(gw.shape)) < 1e-2, ("W", li)
        assert rel(gb, np.asarray(wb).reshape(gb.shape)) < 1e-2, ("b", li)


def _train_setup():
    rng = np.random.default_rng(11)
    n, batch = 2048, 256
    x = rng.normal(0, 1, (n, 64)).astype(np.float32)
    y = (np.tanh(x[:, 0]) * 3 - x[:, 1] ** 2).astype(np.float32)
    order = dg.minibatch_order(n, batch, 2, seed=12)
    return x, y, order, batch


def _flat_oracle_state(params, opt):
    """Oracle parameters and Adam moments as flat arrays in the library's order."""
    p = esc.params_to_flat(params)
    m = esc.params_to_flat([tuple(layer) for layer in opt.m])
    v = esc.params_to_flat([tuple(layer) for layer in opt.v])
    return p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)


def _oracle_after(params, x, y, order, batch, steps, lr=1e-3):
    opt = om.Adam(params, lr=lr)
    p = [(np.asarray(w, np.float32), np.asarray(b, np.float32)) for w, b in params]
    losses = []
    for s in range(steps):
        idx = order[s * batch:(s + 1) * batch]
        yhat, acts = om.forward(p, x[idx])
        losses.append(om.loss(yhat, y[idx]))
        p = opt.step(p, om.backward(p, acts, yhat, y[idx]))
    return p, opt, np.array(losses)


LAYER_SLICES = [slice(0, 64 * 256), slice(64 * 256, 64 * 256 + 256), slice(16640, 16640 + 65536),
                slice(82176, 82176 + 256), slice(82432, 82432 + 65536), slice(147968, 147968 + 256),
                slice(148224, 148224 + 256), slice(148480, 148481)]


def _per_layer_close(got, want, frac):
    """|got - want| <= frac * max|want| within every parameter block."""
    for sl in LAYER_SLICES:
        scale = float(np.max(np.abs(want[sl])))
        assert np.all(np.abs(got[sl] - want[sl]) <= frac * scale + 1e-30), (sl, scale)


@pytest.mark.parametrize("steps", [1, 2])
def test_first_adam_steps_elementwise(ctx, steps):
    """Per element, after one and after two steps: the weights' and biases'
    displacement from the start, and both Adam moments.  Step 1 moves every
    weight by lr * g / (|g| + eps), almost exactly +-lr, whatever the betas;
    step 2 (m = 0.09 g1 + 0.1 g2, v = 0.000999 g1^2 + 0.001 g2^2, bias
    corrections 0.19 and 0.001999) depends on both betas, eps and the bias
    correction.  A float32 replica of the oracle stays within 0.035 lr of
    the oracle's weights and within 1e-4 of each block's largest moment over
    these steps; the GPU sums in another order, so the bounds are looser."""
    import torch
    x, y, order, batch = _train_setup()
    lr = 1e-3
    params = dg.mlp_init(7)
    p0 = esc.params_to_flat(params).astype(np.float64)
    m = esc.MLP(ctx, params)
    m.train(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(order).cuda(), steps, batch,
            lr=lr)
    gp, gm, gv, nsteps = m.get_state()
    assert nsteps == steps
    p_or, opt, _ = _oracle_after(params, x, y, order, batch, steps, lr)
    op, omm, ov = _flat_oracle_state(p_or, opt)
    disp_gpu, disp_or = gp - p0, op - p0
    diff = np.abs(disp_gpu - disp_or)
    assert np.quantile(diff, 0.999) <= 0.05 * lr, np.quantile(diff, 0.999)
    assert diff.max() <= 2.05 * lr * steps          # sign flips of vanishing gradients at most
    if steps == 1:                                  # nearly every weight moved by lr
        assert np.mean(np.abs(np.abs(disp_gpu) - lr) < 0.05 * lr) > 0.95
    _per_layer_close(gm, omm, 1e-2)
    _per_layer_close(gv, ov, 2e-2)


# Largest and 99th-percentile moment differences allowed after 16 steps, as
# fractions of each parameter block's largest moment: about 2.5 times what a
# float32 replica of the oracle shows on this data (m: weights 0.022-0.075 /
# 0.011-0.020, biases 0.055-0.12 / 0.049-0.071; v: at most 0.038 / 0.022).
# b4's first moment sums gradients that cancel (the replica is off by 4.5
# times its size), so it is left out.
M16 = {"W": (0.2, 0.05), "b": (0.3, 0.2)}
V16 = (0.1, 0.06)


def test_sixteen_adam_steps_elementwise(ctx):
    """16 steps (two epochs of 8 batches): per-step losses, and per element the
    weights, biases and both Adam moments against the oracle.  A float32
    replica of the oracle drifts from its weights by 0.05 lr (median), 0.46 lr
    (99th percentile) and 4.3 lr (max) over these steps; the bounds below are
    about twice that."""
    import torch
    x, y, order, batch = _train_setup()
    lr = 1e-3
    params = dg.mlp_init(7)
    m = esc.MLP(ctx, params)
    loss = m.train(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(order).cuda(),
                   len(order) // batch, batch, lr=lr)
    p_or, opt, loss_or = _oracle_after(params, x, y, order, batch, 16, lr)
    assert len(loss) == 16
    assert np.allclose(loss, loss_or, rtol=2e-2, atol=1e-4), (loss, loss_or)
    gp, gm, gv, steps = m.get_state()
    assert steps == 16
    op, omm, ov = _flat_oracle_state(p_or, opt)
    diff = np.abs(gp - op)
    assert np.median(diff) <= 0.15 * lr, np.median(diff)
    assert np.quantile(diff, 0.99) <= 1.0 * lr, np.quantile(diff, 0.99)
    assert diff.max() <= 10 * lr
    for k, sl in enumerate(LAYER_SLICES):
        kind = "W" if k % 2 == 0 else "b"
        if k < 7:
            dm = np.abs(gm[sl] - omm[sl]) / np.max(np.abs(omm[sl]))
            assert dm.max() <= M16[kind][0] and np.quantile(dm, 0.99) <= M16[kind][1], (k, dm.max())
        dv = np.abs(gv[sl] - ov[sl]) / np.max(np.abs(ov[sl]))
        assert dv.max() <= V16[0] and np.quantile(dv, 0.99) <= V16[1], (k, dv.max())
    assert np.mean(loss[-4:]) < np.mean(loss[:4])


def test_training_is_deterministic_and_resumes_exactly(ctx, tmp_path):
    """Two trainings from the same start give bit-identical states; training
    8 steps, saving, loading into a fresh estimator and training 8 more gives
    the same bits (parameters, moments, step count, losses) as 16 steps
    without the interruption.  A damaged checkpoint is refused and leaves the
    estimator unchanged."""
    import torch
    x, y, order, batch = _train_setup()
    xt, yt = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    ot = torch.from_numpy(order).cuda()
    params = dg.mlp_init(7)
    full = esc.MLP(ctx, params)
    loss_full = full.train(xt, yt, ot, 16, batch)
    again = esc.MLP(ctx, params)
    loss_again = again.train(xt, yt, ot, 16, batch)
    for a, b in zip(full.get_state(), again.get_state()):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert np.array_equal(loss_full, loss_again)

    first = esc.MLP(ctx, params)
    loss_a = first.train(xt, yt, ot, 8, batch)
    path = tmp_path / "est.ckpt"
    first.save(path)
    resumed = esc.MLP(ctx)
    resumed.load(path)
    assert resumed.get_state()[3] == 8
    loss_b = resumed.train(xt, yt, ot[8 * batch:].contiguous(), 8, batch)
    for a, b in zip(full.get_state(), resumed.get_state()):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    assert np.array_equal(np.concatenate([loss_a, loss_b]), loss_full)

    raw = bytearray(path.read_bytes())
    raw[200] ^= 1
    bad = tmp_path / "bad.ckpt"
    bad.write_bytes(bytes(raw))
    before = resumed.get_state()
    with pytest.raises(esc.EscError) as ei:
        resumed.load(bad)
    assert ei.value.status == esc.ERR_INVALID and "checksum" in str(ei.value)
    (tmp_path / "short.ckpt").write_bytes(bytes(raw[:1000]))
    with pytest.raises(esc.EscError):
        resumed.load(tmp_path / "short.ckpt")
    for a, b in zip(before, resumed.get_state()):
        assert np.array_equal(np.asarray(a), np.asarray(b))


def test_training_learns(ctx):
    import torch
    rng = np.random.default_rng(13)
    n = 16384
    x = rng.uniform(0, 1, (n, 64)).astype(np.float32)
    y = (np.log(x[:, 2] * x[:, 5] + 1e-3) + x[:, 7]).astype(np.float32)
    order = dg.minibatch_order(n, 1024, 20, seed=14)
    m = esc.MLP(ctx, dg.mlp_init(7))
    loss = m.train(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(order).cuda(),
                   len(order) // 1024, 1024, lr=1e-3)
    # the oracle, trained on the same data and order, ends at 0.1017 of its
    # first loss (0.0484 after 0.4757)
    assert loss[-10:].mean() < 0.15 * loss[:10].mean()
    assert abs(loss[-10:].mean() - 0.0484) < 0.1 * 0.0484
