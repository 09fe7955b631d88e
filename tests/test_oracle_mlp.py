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


# --------------------------------------------------------------------------
# pins of the feature definition (oracle.mlp.features)
# --------------------------------------------------------------------------
import math  # noqa: E402

import oracle  # noqa: E402

RN22 = 0.37416573867739417  # |r| of the CAS(2,2) case below, sqrt(0.1^2 + 1e-9^2 + 0.2^2 + 0.3^2)


def test_features_hand_computed_cas22():
    """CAS(2e,2o), one electron of each spin: strings 01, 10 for both spins, so the
    determinants are (01,01), (01,10), (10,01), (10,10). theta = 2, d_min = 1.
    The second determinant sits exactly at d = theta (the clamp takes +1e-8),
    the third 5e-9 below it (the clamp takes -1e-8). Every value below was
    worked out by hand from the definitions (N = 4, sqrt N = 2)."""
    astr = oracle.strings(2, 1)
    bstr = oracle.strings(2, 1)
    d = np.array([1.0, 2.0, 2.0 - 5e-9, 3.0])
    r = np.array([0.1, 1e-9, -0.2, 0.3])
    x = np.array([0.5, -0.5, 0.25, 0.75])
    F = mlp.features(d, 2.0, r, x, astr, bstr, 2, 1, 1, 1.0)
    expect = np.array([
        # f0 tanh(-1/4)   f1 asinh(0.2/|r|)      f2 asinh(1)         f3 asinh(0.1*2/|r|)  f4  f5  f6  f7
        [-0.24491866240370913, 0.5118746150936737, 0.881373587019543, 0.5118746150936737, 0.0, 0.0, 0.0, 0.0],
        # d = theta: f0 = 0; f3 = asinh(-1e-9/1e-8 * 2/|r|); beta string 10 has its electron outside
        # orbital 0; the two strings differ in both orbitals; f7 = tanh(1/4)
        [0.0, 5.345224838248488e-09, -0.881373587019543, -0.5118746150936737, 0.0, 1.0, 1.0,
         0.24491866240370913],
        # d - theta = -5e-9: f0 = tanh(-1.25e-9); f3 = asinh(-(-0.2)/(-1e-8) * 2/|r|)
        [-1.25e-09, -0.9293629477662251, 0.48121182505960347, -19.18059362082457, 1.0, 0.0, 1.0,
         0.2449186612286906],
        # d - theta = 1: f3 = asinh(-0.3 * 2/|r|); both strings excited, identical
        [0.24491866240370913, 1.2508725589454122, 1.1947632172871094, -1.2508725589454122, 1.0, 1.0, 0.0,
         0.46211715726000974],
    ])
    np.testing.assert_allclose(F, expect, rtol=1e-13, atol=1e-16)


def _case(n, na, nb, seed):
    rng = np.random.default_rng(seed)
    astr = oracle.strings(n, na)
    bstr = oracle.strings(n, nb)
    N = astr.size * bstr.size
    d = rng.uniform(-3.0, 3.0, N)
    theta = float(d[N // 3]) + 0.3
    r = rng.normal(size=N)
    x = rng.normal(size=N) / math.sqrt(N)
    dmin = float(d.min())
    F = mlp.features(d, theta, r, x, astr, bstr, n, na, nb, dmin)
    return astr, bstr, N, d, theta, r, x, dmin, F


@pytest.mark.parametrize("n,na,nb,seed", [(4, 2, 2, 1), (5, 3, 2, 2)])
def test_features_invert_to_their_inputs(n, na, nb, seed):
    """Each continuous feature is an invertible map of its input: undoing it
    recovers d, r, x and the diagonal correction (a change of a scale, a sign or
    a normalisation in any of them breaks one of these)."""
    astr, bstr, N, d, theta, r, x, dmin, F = _case(n, na, nb, seed)
    rn = np.linalg.norm(r)
    np.testing.assert_allclose(4.0 * np.arctanh(F[:, 0]) + theta, d, atol=1e-12)
    np.testing.assert_allclose(np.sinh(F[:, 1]) * rn / math.sqrt(N), r, atol=1e-12)
    np.testing.assert_allclose(np.sinh(F[:, 2]) / math.sqrt(N), x, atol=1e-13)
    np.testing.assert_allclose(np.sinh(F[:, 3]) * rn / math.sqrt(N), -r / (d - theta), rtol=1e-11)
    np.testing.assert_allclose(4.0 * np.arctanh(F[:, 7]) + dmin, d, atol=1e-12)
    i0 = int(np.argmin(d))
    assert F[i0, 7] == 0.0  # the lowest diagonal element
    # f1 and f3 change sign with the residual
    F2 = mlp.features(d, theta, -r, x, astr, bstr, n, na, nb, dmin)
    np.testing.assert_allclose(F2[:, 1], -F[:, 1], atol=0)
    np.testing.assert_allclose(F2[:, 3], -F[:, 3], atol=0)


def test_occupation_features_by_hand():
    """CAS(5,5) with 3 alpha and 2 beta electrons. Strings ascending:
    alpha 7, 11, 13, 14, 19, 21, 22, 25, 26, 28 have 0,1,1,1,1,1,1,2,2,2 electrons
    in orbitals 3-4 (outside the lowest 3), divided by min(3, 2) = 2; beta 3, 5,
    6, 9, 10, 12, 17, 18, 20, 24 have 0,1,1,1,1,2,1,1,2,2 electrons outside the
    lowest 2, divided by min(2, 3) = 2."""
    astr, bstr, N, d, theta, r, x, dmin, F = _case(5, 3, 2, 3)
    assert astr.tolist() == [7, 11, 13, 14, 19, 21, 22, 25, 26, 28]
    assert bstr.tolist() == [3, 5, 6, 9, 10, 12, 17, 18, 20, 24]
    f4 = np.array([0, 1, 1, 1, 1, 1, 1, 2, 2, 2]) / 2.0
    f5 = np.array([0, 1, 1, 1, 1, 2, 1, 1, 2, 2]) / 2.0
    G = F.reshape(10, 10, 8)
    np.testing.assert_array_equal(G[:, :, 4], np.repeat(f4[:, None], 10, axis=1))
    np.testing.assert_array_equal(G[:, :, 5], np.repeat(f5[None, :], 10, axis=0))
    # open-shell fraction: popcount(Ia xor Ib) / 5 for a few pairs worked by hand
    # 7 ^ 3 = 4 (one bit); 28 ^ 3 = 31 (five); 11 ^ 9 = 2 (one); 14 ^ 12 = 2 (one); 13 ^ 5 = 8 (one);
    # 25 ^ 24 = 1 (one); 21 ^ 20 = 1; 22 ^ 6 = 16 (one); 26 ^ 18 = 8; 19 ^ 17 = 2; 28 ^ 12 = 16
    for ia, ib, bits in [(0, 0, 1), (9, 0, 5), (1, 3, 1), (3, 5, 1), (2, 1, 1), (7, 9, 1), (5, 8, 1),
                         (6, 2, 1), (8, 7, 1), (4, 6, 1), (9, 5, 1), (0, 9, 5)]:
        assert G[ia, ib, 6] == bits / 5.0, (ia, ib)


def test_aufbau_and_closed_shell_values():
    """f4 = f5 = 0 on the aufbau strings, f6 = 0 when the alpha and beta strings
    are equal, f0 = 0 where H_II = theta."""
    n, na, nb = 4, 2, 2
    astr = oracle.strings(n, na)
    bstr = oracle.strings(n, nb)
    Na, Nb = astr.size, bstr.size
    rng = np.random.default_rng(9)
    d = rng.uniform(-1, 1, Na * Nb)
    theta = float(d[7])
    F = mlp.features(d, theta, rng.normal(size=Na * Nb), rng.normal(size=Na * Nb), astr, bstr, n, na, nb,
                     float(d.min())).reshape(Na, Nb, 8)
    assert np.all(F[0, :, 4] == 0) and np.all(F[:, 0, 5] == 0)
    assert np.all(F[1:, :, 4] > 0) and np.all(F[:, 1:, 5] > 0)
    for i in range(Na):
        assert F[i, i, 6] == 0.0
    assert F.reshape(-1, 8)[7, 0] == 0.0


@pytest.mark.parametrize("n,na,nb,div_a,div_b", [(6, 4, 1, 2, 1), (6, 1, 4, 1, 2)])
def test_excitation_features_divisors(n, na, nb, div_a, div_b):
    """Unequal electron counts: the alpha level is divided by min(n_a, n - n_a)
    and the beta level by min(n_b, n - n_b) (worked out: 2 and 1, or 1 and 2)."""
    astr, bstr, N, d, theta, r, x, dmin, F = _case(n, na, nb, 4)
    G = F.reshape(astr.size, bstr.size, 8)
    outside = lambda m, ne: sum(1 for p in range(ne, n) if (int(m) >> p) & 1)  # noqa: E731
    for i, m in enumerate(astr):
        assert np.all(G[i, :, 4] * div_a == outside(m, na))
    for j, m in enumerate(bstr):
        assert np.all(G[:, j, 5] * div_b == outside(m, nb))


def test_diagonal_correction_clamp_boundary():
    """|d - theta| is clamped to 1e-8 with its sign, and only below 1e-8: the
    denominators of d - theta = 5e-7, -5e-7, 2e-8, 5e-9, -5e-9 are 5e-7, -5e-7,
    2e-8, 1e-8 and -1e-8."""
    astr = oracle.strings(2, 1)
    theta = 0.5
    gaps = np.array([5e-7, -5e-7, 2e-8, 5e-9])
    for last in (5e-9, -5e-9):
        g = gaps.copy()
        g[3] = last
        d = theta + g
        den = np.array([5e-7, -5e-7, 2e-8, 1e-8 if last > 0 else -1e-8])
        r = np.array([0.3, -0.1, 0.2, 0.4])
        F = mlp.features(d, theta, r, np.ones(4) / 2, astr, astr, 2, 1, 1, float(d.min()))
        rn = np.linalg.norm(r)
        np.testing.assert_allclose(np.sinh(F[:, 3]) * rn / 2.0, -r / den, rtol=1e-9)
