"""CPU oracle of the learned cardinality estimator (numpy, float64).

TEST INFRASTRUCTURE ONLY: used by tests and the smoke check, never by the
product path.

The paper replaces synopses with an exact count (Section 2, Section 2.4);
the learned gate that decides which predicates deserve that exact count is
this build's extension, so its definition is the one written out here:

  network   64 -> 256 -> 256 -> 256 -> 1, ReLU after each hidden layer,
            weights stored [fan_in, fan_out], output = ln(selectivity);
  rounding  every matrix-product operand is rounded to bfloat16
            (round-to-nearest-even): the input X, the weights, the hidden
            activations handed to the next layer, and the back-propagated
            deltas handed to a product; sums are exact in float64 here;
  loss      L = mean_b h(yhat_b - y_b), the Huber loss with threshold
            d = 1/2: h(e) = e^2 / 2 for |e| <= d, d (|e| - d / 2) beyond
            (its derivative is e clamped to [-d, d]);
  backward  chain rule; the ReLU derivative is 1 where the (rounded)
            activation is > 0 and 0 elsewhere (0 at exactly 0); bias
            gradients sum the un-rounded deltas;
  update    Adam (Kingma and Ba) on float32 master weights:
            m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
            w -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).

With rounding=False the same code is the exact float64 network, which the
tests pin against central finite differences.
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if nan.any():
        out[nan] = np.nan
    return out


def _id(x):
    return np.asarray(x, dtype=np.float64)


def forward(params, x, rounding=True):
    """Returns (yhat, cache).  params = [(W1,b1), ..., (W4,b4)]."""
    r = bf16 if rounding else _id
    a = r(x)
    acts = [a]
    nl = len(params)
    for i, (w, b) in enumerate(params):
        z = a @ r(w) + np.asarray(b, np.float64)
        if i == nl - 1:
            return z[:, 0], acts
        h = np.maximum(z, 0.0)
        a = r(h)
        acts.append(a)
    raise AssertionError


HUBER = 0.5


def loss(yhat, y):
    e = np.asarray(yhat, np.float64) - np.asarray(y, np.float64)
    a = np.abs(e)
    return float(np.mean(np.where(a <= HUBER, 0.5 * e * e, HUBER * (a - 0.5 * HUBER))))


def backward(params, acts, yhat, y, rounding=True):
    """Gradients [(dW1, db1), ...] of the mean Huber loss."""
    r = bf16 if rounding else _id
    bsz = len(y)
    d = np.clip(yhat - np.asarray(y, np.float64), -HUBER, HUBER) / bsz   # dL/dyhat, shape [B]
    grads = [None] * len(params)
    # output layer: yhat = a3 . w4 + b4
    w4 = params[-1][0]
    grads[-1] = (acts[-1].T @ d[:, None], np.array([d.sum()]))
    dh = d[:, None] @ r(w4).T                                    # [B, 256]
    for i in range(len(params) - 2, -1, -1):
        dz = dh * (acts[i + 1] > 0)
        g = r(dz)
        grads[i] = (acts[i].T @ g, dz.sum(axis=0))
        if i > 0:
            dh = g @ r(params[i][0]).T
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros(np.shape(a), np.float64) for a in layer] for layer in params]
        self.v = [[np.zeros(np.shape(a), np.float64) for a in layer] for layer in params]

    def step(self, params, grads):
        """One update; returns new float32 (W, b) pairs."""
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (layer, glayer) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(zip(layer, glayer)):
                g = np.asarray(g, np.float64).reshape(np.shape(p))
                self.m[i][j] = self.b1 * self.m[i][j] + (1.0 - self.b1) * g
                self.v[i][j] = self.b2 * self.v[i][j] + (1.0 - self.b2) * g * g
                upd = self.lr * (self.m[i][j] / c1) / (np.sqrt(self.v[i][j] / c2) + self.eps)
                new.append((np.asarray(p, np.float64) - upd).astype(np.float32))
            out.append(tuple(new))
        return out


def train(params, x, y, order, batch, lr=1e-3, rounding=True):
    """Minibatch Adam over the sample order `order` (len multiple of batch)."""
    opt = Adam(params, lr=lr)
    p = [(np.asarray(w, np.float32), np.asarray(b, np.float32)) for w, b in params]
    losses = []
    for s in range(len(order) // batch):
        idx = order[s * batch:(s + 1) * batch]
        yhat, acts = forward(p, x[idx], rounding)
        losses.append(loss(yhat, y[idx]))
        p = opt.step(p, backward(p, acts, yhat, y[idx], rounding))
    return p, losses


def q_error(c_hat, c, n):
    """q = max(c'/c_hat, c_hat/c') with c' = max(c, 1) and c_hat clamped to [1, n]."""
    c_hat = np.clip(np.asarray(c_hat, np.float64), 1.0, float(n))
    cp = np.maximum(np.asarray(c, np.float64), 1.0)
    return np.maximum(c_hat / cp, cp / c_hat)


def label(c, n):
    """Training target: y = ln(max(c, 1) / n)."""
    return np.log(np.maximum(np.asarray(c, np.float64), 1.0) / float(n))
