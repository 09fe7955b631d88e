"""Pins of the FP64 MLP oracle: finite differences and closed-form special cases."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.normal(size=(37, mlp.D_IN))
    T = rng.normal(size=37)
    L, g = mlp.loss_and_grad(p, X, T)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 120, replace=False), [mlp.NPARAM - 1, 0, 512, 4700]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, T)[0] - mlp.loss_and_grad(p - e, X, T)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_zero_hidden_weights_closed_form():
    """W1 = W2 = 0: every hidden unit is tanh of its bias, so y = b3 + W3 . tanh(b2)."""
    rng = np.random.default_rng(2)
    p = np.zeros(mlp.NPARAM)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    o = mlp.D_IN * mlp.H
    p[o:o + mlp.H] = rng.normal(size=mlp.H)            # b1 (irrelevant: W2 = 0)
    o2 = o + mlp.H + mlp.H * mlp.H
    b2v = rng.normal(size=mlp.H)
    p[o2:o2 + mlp.H] = b2v
    w3 = rng.normal(size=mlp.H)
    p[o2 + mlp.H:o2 + 2 * mlp.H] = w3
    p[-1] = 0.3
    X = rng.normal(size=(5, mlp.D_IN))
    np.testing.assert_allclose(mlp.forward(p, X), 0.3 + w3 @ np.tanh(b2v), rtol=0, atol=1e-14)


def test_single_path_network():
    """Only W1[k][0], W2[0][0], W3[0] nonzero: y = w3 tanh(w2 tanh(w1 x_k))."""
    p = np.zeros(mlp.NPARAM)
    k = 3
    p[k * mlp.H + 0] = 0.7                                # W1[3][0]
    p[mlp.D_IN * mlp.H + mlp.H + 0] = -1.3                # W2[0][0]
    p[mlp.D_IN * mlp.H + mlp.H + mlp.H * mlp.H + mlp.H + 0] = 2.0   # W3[0]
    X = np.linspace(-2, 2, 9)[:, None] * np.eye(mlp.D_IN)[k][None, :]
    ref = 2.0 * np.tanh(-1.3 * np.tanh(0.7 * X[:, k]))
    np.testing.assert_allclose(mlp.forward(p, X), ref, rtol=0, atol=1e-14)
