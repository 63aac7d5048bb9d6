"""FP64 reference of the overlap-weight network (oracle; test infrastructure).

Not part of the paper: the library can replace the fixed face-centred normal
weights of Sec. 3.1 (eq. (weight function:fc)) by a learned transition width
theta and damping omega per face, predicted by a small MLP.  This module is
the plain numpy definition the GPU kernels are checked against.

Network: x (D_IN) -> tanh(W1 x + b1) (H) -> tanh(W2 h1 + b2) (H) -> W3 h2 + b3 (D_OUT).
Parameter vector layout: W1 (H x D_IN, row-major), b1, W2 (H x H), b2,
W3 (D_OUT x H), b3.
Loss: L = (1/B) sum_b sum_o (y_bo - t_bo)^2.
Adam (Kingma & Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Pins (tests/test_oracle_mlp.py): gradients against central finite
differences, a zero-weight closed form, one Adam step in closed form.
"""
from __future__ import annotations

import numpy as np

D_IN, H, D_OUT = 6, 64, 2
N_PARAMS = H * D_IN + H + H * H + H + D_OUT * H + D_OUT


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D_IN].reshape(H, D_IN); o += H * D_IN
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + D_OUT * H].reshape(D_OUT, H); o += D_OUT * H
    b3 = p[o:o + D_OUT]; o += D_OUT
    assert o == N_PARAMS
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def init(seed=0):
    """Deterministic init: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.uniform(-1, 1, (H, D_IN)) / np.sqrt(D_IN)
    W2 = rng.uniform(-1, 1, (H, H)) / np.sqrt(H)
    W3 = rng.uniform(-1, 1, (D_OUT, H)) / np.sqrt(H)
    return pack(W1, np.zeros(H), W2, np.zeros(H), W3, np.zeros(D_OUT))


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y, (X, h1, h2)


def loss(p, X, T):
    y, _ = forward(p, X)
    return float(np.sum((y - T) ** 2) / len(X))


def grad(p, X, T):
    """dL/dp by backpropagation (chain rule through tanh: 1 - h^2)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    y, (X, h1, h2) = forward(p, X)
    B = len(X)
    dy = 2.0 * (y - T) / B
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    da2 = (dy @ W3) * (1.0 - h2 ** 2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * (1.0 - h1 ** 2)
    gW1 = da1.T @ X
    gb1 = da1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
