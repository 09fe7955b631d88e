"""Learned preconditioner on the GPU: forward, gradients and features against
the FP64 oracle, training, Davidson with the network and its Olsen fallback,
and the measured gain over the method without it."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from paper_2405_10197_amd import casci, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def params(seed, scale=1.0):
    rng = np.random.default_rng(seed + 100)
    p = omlp.init_params(seed) * scale
    p[:] += rng.normal(0, 0.02, p.size)   # nonzero biases too
    return p.astype(np.float32)


def test_forward_matches_oracle(torch):
    c = casci.Context(0)
    p = params(3)
    c.mlp_set_params(p)
    X = np.random.default_rng(4).normal(size=(3000, 8)).astype(np.float32)
    y = c.mlp_forward(X)
    ref = omlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.abs(y - ref).max() < 2e-5 * max(1.0, np.abs(ref).max())


def test_loss_gradient_matches_oracle(torch):
    c = casci.Context(0)
    p = params(5)
    c.mlp_set_params(p)
    rng = np.random.default_rng(6)
    X = rng.normal(size=(5000, 8)).astype(np.float32)
    T = rng.normal(size=5000).astype(np.float32)
    L, g = c.mlp_loss_grad(X, T)
    Lo, go = omlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert abs(L - Lo) < 1e-5 * Lo
    assert np.abs(g - go).max() < 1e-4 * np.abs(go).max()


def test_training_fits_a_teacher_network(torch):
    c = casci.Context(0)
    rng = np.random.default_rng(7)
    X = rng.normal(size=(20000, 8)).astype(np.float32)
    T = omlp.forward(params(8).astype(np.float64), X.astype(np.float64)).astype(np.float32)
    c.mlp_set_params(params(9))
    L0, _ = c.mlp_loss_grad(X, T)
    hist = c.mlp_train(X, T, epochs=30, batch=1024, lr=3e-3, seed=1)
    L1, _ = c.mlp_loss_grad(X, T)
    assert np.all(np.isfinite(hist))
    assert L1 < 0.05 * L0, (L0, L1, hist[-5:])


def test_features_match_oracle(torch):
    n, na, nb = 6, 3, 3
    h, eri, _ = synth.integrals(n, 1)
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(na, nb, n)
    d = c.dims
    x = synth.ci_vector(d["Na"], d["Nb"], 3)[0]
    xt = torch.from_numpy(x).cuda()
    sx = c.sigma(xt)
    theta = float((xt * sx).sum().item())
    idx = np.arange(d["Ndet"])
    F = c.mlp_features(xt, sx, theta, idx)
    diag = np.diag(oracle.hamiltonian(h, eri, na, nb))
    r = (oracle.sigma(h, eri, na, nb, x) - theta * x).ravel()
    Fo = omlp.features(diag, theta, r, x.ravel(), oracle.strings(n, na), oracle.strings(n, nb), n, na, nb,
                       diag.min())
    assert np.abs(F - Fo).max() < 2e-5 * max(1.0, np.abs(Fo).max())


def diag_like_params():
    """A single path W1[3][0] -> W2[0][0] -> W3[0] in the near-linear range of
    tanh, so that the output approximately equals feature f3, the (asinh-
    compressed) diagonal correction."""
    p = np.zeros(omlp.NPARAM)
    H, D = omlp.H, omlp.D_IN
    p[3 * H + 0] = 0.05
    p[D * H + H + 0] = 0.1
    p[D * H + H + H * H + H + 0] = 200.0
    return p.astype(np.float32)


def test_mlp_davidson_converges_and_falls_back(torch):
    n, na, nb, k = 8, 4, 4, 3
    h, eri, _ = synth.integrals(n, 3000)
    Eo, _, _ = oracle.solve(h, eri, na, nb, nroots=k)
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(na, nb, n)
    c.mlp_set_params(diag_like_params())
    E, _, info = c.davidson(k, 1e-11, precond="mlp", r_tol=1e-7, vectors=False, max_iter=400)
    assert info["converged"] and info["mlp_fallbacks"] == 0
    assert np.abs(E - Eo).max() < 1e-10
    bad = np.full(omlp.NPARAM, np.nan, dtype=np.float32)
    c.mlp_set_params(bad)
    E2, _, info2 = c.davidson(k, 1e-11, precond="mlp", r_tol=1e-7, vectors=False)
    assert info2["converged"] and info2["mlp_fallbacks"] > 0
    assert np.abs(E2 - Eo).max() < 1e-10


def test_learned_preconditioner_gain_cas10(torch):
    """Train on residual -> converged-correction pairs from CAS(10,10) solves of
    four seeds of the integral family, then solve a held-out seed: report the
    iteration counts of Olsen and of the trained network (both must converge
    to the same energies; the gain itself is measured, not assumed)."""
    n, k = 10, 3
    Fs, Ts = [], []
    for seed in (4100, 4101, 4102, 4103):
        h, eri, _ = synth.integrals(n, seed)
        c = casci.Context(0)
        c.set_integrals(h, eri)
        c.build_strings(5, 5, n)
        d = c.dims
        xs = torch.empty((k, d["Na"], d["Nb"]), dtype=torch.float64, device="cuda")
        E, _, info = c.davidson(k, 1e-12, precond="olsen", r_tol=1e-8, vectors_out=xs)
        assert info["converged"]
        F, T = c.mlp_collect(k, 1e-10, xs, samples=2048, seed=seed, precond="olsen")
        Fs.append(F)
        Ts.append(T)
    F = torch.cat(Fs).contiguous()
    T = torch.cat(Ts).contiguous()
    assert F.shape[0] > 10000 and bool(torch.isfinite(F).all()) and bool(torch.isfinite(T).all())
    h, eri, _ = synth.integrals(n, 4104)
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(5, 5, n)
    c.mlp_set_params(params(12))
    hist = c.mlp_train(F, T, epochs=20, batch=4096, lr=2e-3, seed=3)
    assert hist[-1] < hist[0]
    E0, _, i0 = c.davidson(k, 1e-10, precond="olsen", vectors=False, max_iter=400)
    E1, _, i1 = c.davidson(k, 1e-10, precond="mlp", vectors=False, max_iter=400)
    print("\n[gain] CAS(10,10) held-out seed: Olsen %d iterations / %d sigma; learned %d iterations / %d sigma "
          "(%d fallbacks); training loss %.3f -> %.3f" % (i0["iterations"], i0["sigma_calls"], i1["iterations"],
                                                          i1["sigma_calls"], i1["mlp_fallbacks"], hist[0], hist[-1]))
    assert i0["converged"] and i1["converged"]
    assert np.abs(E1 - E0).max() < 1e-8
