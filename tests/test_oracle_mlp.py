"""Pins of the FP64 MLP reference: finite differences and closed forms."""
import numpy as np
import pytest

from oracle import mlp


def test_param_count_and_roundtrip():
    p = mlp.init(1)
    assert len(p) == mlp.N_PARAMS == 6 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2
    assert np.array_equal(mlp.pack(*mlp.unpack(p)), p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init(2) + 0.05 * rng.standard_normal(mlp.N_PARAMS)
    X = rng.standard_normal((7, mlp.D_IN))
    T = rng.standard_normal((7, mlp.D_OUT))
    g = mlp.grad(p, X, T)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), i


def test_zero_weights_closed_form():
    p = np.zeros(mlp.N_PARAMS)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p.copy())
    b3 = np.array([0.3, -0.2])
    p = mlp.pack(W1, b1, W2, b2, W3, b3)
    X = np.ones((4, mlp.D_IN))
    T = np.array([[1.0, 0.0]] * 4)
    y, _ = mlp.forward(p, X)
    assert np.allclose(y, b3)
    g = mlp.grad(p, X, T)
    gb3 = mlp.unpack(g)[5]
    assert np.allclose(gb3, 2 * (b3 - T[0]))            # mean over the batch of 2 (y - t)
    assert np.allclose(mlp.unpack(g)[4], 0.0)           # h2 = 0 -> no W3 gradient


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    lr, eps = 1e-2, 1e-8
    p1, m, v = mlp.adam_step(p, g, np.zeros(10), np.zeros(10), 1, lr=lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
