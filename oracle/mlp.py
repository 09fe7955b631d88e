"""FP64 oracle of the learned Davidson preconditioner -- TEST INFRASTRUCTURE ONLY.

The network maps 8 per-determinant features to one output:
    z1 = x W1 + b1,  a1 = tanh(z1)       (8 -> 64)
    z2 = a1 W2 + b2, a2 = tanh(z2)       (64 -> 64)
    y  = a2 W3 + b3                      (64 -> 1)
Loss over a batch of N samples: L = (1/N) sum_i (y_i - t_i)^2.

Parameter vector layout (4801 values): W1[8][64] row-major (input, unit),
b1[64], W2[64][64], b2[64], W3[64], b3[1].

Features of determinant I = (Ia, Ib) for a Ritz pair (theta, x) with residual
r = H x - theta x (d = H_II, N = number of determinants):
    f0 = tanh((d - theta) / 4)
    f1 = asinh(r_I sqrt(N) / |r|)
    f2 = asinh(x_I sqrt(N))
    f3 = asinh(-r_I / (d - theta) * sqrt(N) / |r|)   (|d - theta| clamped >= 1e-8)
    f4 = (alpha electrons outside the lowest n_alpha orbitals) / max(1, min(n_alpha, n - n_alpha))
    f5 = the same for beta
    f6 = popcount(Ia xor Ib) / n          (open-shell fraction)
    f7 = tanh((d - d_min) / 4)            (d_min = lowest diagonal element)
Training target for iteration k of a solve converging to x*:
    t_I = (x* - x_k)_I sqrt(N) / |x* - x_k|, with x* signed so that x* . x_k > 0.

Pins (tests): finite differences of the loss for the gradient, special
weights for which the network reduces to closed forms, and for the features:
rows of a CAS(2,2) case worked out by hand (including both signs of the
clamp), the inverse maps that recover d, r, x and -r/(d - theta) from
f0..f3 and f7, excitation counts and open-shell fractions of hand-listed
strings with unequal divisors, and the clamp boundary.
"""
from __future__ import annotations

import math

import numpy as np

D_IN, H = 8, 64
NPARAM = D_IN * H + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    if p.size != NPARAM:
        raise ValueError("expected %d parameters" % NPARAM)
    o = 0
    W1 = p[o:o + D_IN * H].reshape(D_IN, H); o += D_IN * H
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, W3, b3


def init_params(seed: int = 0):
    """Scaled Gaussian initialisation (std 1/sqrt(fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, 1 / math.sqrt(D_IN), (D_IN, H))
    W2 = rng.normal(0, 1 / math.sqrt(H), (H, H))
    W3 = rng.normal(0, 1 / math.sqrt(H), H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3, [0.0]])


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    a1 = np.tanh(X @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    return a2 @ W3 + b3


def loss_and_grad(p, X, T):
    """Mean squared error and its gradient, by hand-written backpropagation."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    N = X.shape[0]
    a1 = np.tanh(X @ W1 + b1)
    a2 = np.tanh(a1 @ W2 + b2)
    y = a2 @ W3 + b3
    e = y - T
    L = float(np.mean(e * e))
    dy = 2.0 * e / N
    gW3 = a2.T @ dy
    gb3 = dy.sum()
    dz2 = np.outer(dy, W3) * (1.0 - a2 * a2)
    gW2 = a1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (1.0 - a1 * a1)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, [gb3]])
    return L, g


def features(d, theta, r, x, astr, bstr, n, nalpha, nbeta, dmin):
    """Features of every determinant (see module doc). d, r, x: [Na*Nb]."""
    d = np.asarray(d, dtype=np.float64).ravel()
    r = np.asarray(r, dtype=np.float64).ravel()
    x = np.asarray(x, dtype=np.float64).ravel()
    N = d.size
    rn = np.linalg.norm(r)
    den = d - theta
    den = np.where(np.abs(den) < 1e-8, np.where(den < 0, -1e-8, 1e-8), den)
    sq = math.sqrt(N)
    Nb = len(bstr)
    ia = np.arange(N) // Nb
    ib = np.arange(N) % Nb
    A = np.array([int(s) for s in astr], dtype=object)
    B = np.array([int(s) for s in bstr], dtype=object)
    aufa = (1 << nalpha) - 1
    aufb = (1 << nbeta) - 1
    exa = np.array([bin(int(A[i]) & ~aufa).count("1") for i in range(len(A))])
    exb = np.array([bin(int(B[i]) & ~aufb).count("1") for i in range(len(B))])
    open_ = np.array([[bin(int(A[i]) ^ int(B[j])).count("1") for j in range(len(B))] for i in range(len(A))]).ravel()
    F = np.empty((N, 8))
    F[:, 0] = np.tanh((d - theta) / 4.0)
    F[:, 1] = np.arcsinh(r * sq / rn) if rn > 0 else 0.0
    F[:, 2] = np.arcsinh(x * sq)
    F[:, 3] = np.arcsinh(-r / den * sq / rn) if rn > 0 else 0.0
    F[:, 4] = exa[ia] / max(1, min(nalpha, n - nalpha))
    F[:, 5] = exb[ib] / max(1, min(nbeta, n - nbeta))
    F[:, 6] = open_ / n
    F[:, 7] = np.tanh((d - dmin) / 4.0)
    return F
