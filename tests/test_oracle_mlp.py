"""Pins of the selector network's CPU oracle: closed forms and finite differences."""
import math

import numpy as np

from oracle import mlp


def _data(g, B=37):
    X = g.standard_normal((B, mlp.NF))
    y = g.integers(0, 2, B)
    w = g.random(B) + 0.1
    return X, y, w


def test_parameter_count():
    assert mlp.NPARAMS == 4738


def test_equal_logits_give_log_two():
    g = np.random.default_rng(1)
    X, y, w = _data(g)
    p = np.zeros(mlp.NPARAMS)
    assert abs(mlp.loss(p, X, y, w) - np.mean(w) * math.log(2.0)) < 1e-15


def test_output_bias_only_closed_form():
    g = np.random.default_rng(2)
    X, _, _ = _data(g, 5)
    q = mlp.unpack(np.zeros(mlp.NPARAMS))
    q["b3"] = np.array([1.0, 2.0])
    p = mlp.pack(q)
    y = np.zeros(5, dtype=int)
    w = np.ones(5)
    assert abs(mlp.loss(p, X, y, w) - math.log(1.0 + math.e)) < 1e-14
    assert np.all(mlp.decide(p, X) == 1)


def test_gradient_against_central_differences():
    g = np.random.default_rng(3)
    X, y, w = _data(g)
    p = mlp.init_params(g) + 0.05 * g.standard_normal(mlp.NPARAMS)
    an = mlp.grad(p, X, y, w)
    idx = g.choice(mlp.NPARAMS, 300, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAMS)
        e[k] = h
        fd = (mlp.loss(p + e, X, y, w) - mlp.loss(p - e, X, y, w)) / (2 * h)
        assert abs(fd - an[k]) <= 1e-7 + 1e-5 * abs(fd), k


def test_adam_first_step_is_a_signed_lr_step():
    g = np.random.default_rng(4)
    p = g.standard_normal(mlp.NPARAMS)
    gr = g.standard_normal(mlp.NPARAMS)
    z = np.zeros(mlp.NPARAMS)
    p1, m, v = mlp.adam(p, z, z, gr, 1, lr=1e-3, eps=0.0)
    assert np.allclose(p1, p - 1e-3 * np.sign(gr), rtol=0, atol=1e-15)
