"""CPU oracle of the strategy selector's network: TEST INFRASTRUCTURE ONLY.

A 6-64-64-2 perceptron with ReLU hidden layers, trained with a per-sample
weighted softmax cross-entropy and Adam, all in binary64 NumPy.  Parameters are
one flat vector in the order W1 [64x6], b1 [64], W2 [64x64], b2 [64],
W3 [2x64], b3 [2] (weights row-major, output x input): 4738 values.

Loss of a batch of B samples (features x_b, label y_b in {0, 1}, weight w_b):
    L = (1/B) * sum_b  w_b * ( logsumexp(z_b) - z_b[y_b] ),   z_b = the two logits.
Adam (Kingma & Ba, 2015):  m <- b1 m + (1-b1) g,  v <- b2 v + (1-b2) g^2,
    p <- p - lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

NF, NH, NO = 6, 64, 2
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NO, NH)), ("b3", (NO,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(p[k:k + size], dtype=np.float64).reshape(shape)
        k += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(g: np.random.Generator):
    """He-style initialisation (drawn here, passed to both sides as input)."""
    parts = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            parts[name] = g.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            parts[name] = np.zeros(shape)
    return pack(parts)


def forward(p, X):
    q = unpack(p)
    z1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ q["W3"].T + q["b3"]
    return z3, (z1, h1, z2, h2)


def loss(p, X, y, w):
    z, _ = forward(p, X)
    zmax = np.max(z, axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(np.sum(np.exp(z - zmax), axis=1))
    return float(np.mean(w * (lse - z[np.arange(len(y)), y])))


def grad(p, X, y, w):
    """Gradient of ``loss`` by backpropagation."""
    q = unpack(p)
    z, (z1, h1, z2, h2) = forward(p, X)
    B = X.shape[0]
    zmax = np.max(z, axis=1, keepdims=True)
    e = np.exp(z - zmax)
    prob = e / np.sum(e, axis=1, keepdims=True)
    onehot = np.zeros_like(prob)
    onehot[np.arange(B), y] = 1.0
    dz3 = (w[:, None] / B) * (prob - onehot)
    g = {"W3": dz3.T @ h2, "b3": dz3.sum(0)}
    dz2 = (dz3 @ q["W3"]) * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ q["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(0)
    return pack(g)


def adam(p, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def decide(p, X):
    """1 (rebuild) where the second logit is larger, else 0 (repair)."""
    z, _ = forward(p, X)
    return (z[:, 1] > z[:, 0]).astype(np.int32)
