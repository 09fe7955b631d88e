"""Parity at the sizes the benchmark runs, through the C ABI.

* Strings and single-substitution lists at CAS(16,16) and CAS(18,18),
  bit-exact against the oracle's operator-by-operator construction.
* Rows of the same-spin operator at n = 16 against the oracle's explicit H of
  the (8, 0) system.
* The sigma path the Davidson solver takes when nalpha = nbeta (one same-spin
  gather for both spins, transposition-parity combination with the
  alpha-beta term), in FP64, FP32 and BF16 alpha-beta arithmetic: whole
  vectors against the oracle on small spaces, sampled rows (first, last, the
  edges of the 32-row tiles of the combination pass, random) at CAS(16,16).
* Invariants that fix the energy at sizes with no explicit matrix: the
  zero-ERI ground state at CAS(16,16), invariance under an orthogonal
  rotation of the orbitals and integral S(S+1) at CAS(12,12).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2405_10197_amd import casci, synth

pytestmark = pytest.mark.gpu

# error bounds of the low-precision alpha-beta arithmetic (relative to max |sigma|):
# FP32 inputs (unit roundoff 2^-24) and BF16 inputs (2^-9 with round-to-nearest),
# both with FP32 accumulation, as in the smaller-space tests
TOL = {"f64": 1e-12, "f32": 2e-6, "bf16": 2e-2}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def make(n, na, nb, seed):
    h, eri, _ = synth.integrals(n, seed)
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(na, nb, n)
    return c, h, eri


@pytest.mark.parametrize("n,ne", [(16, 8), (18, 9)])
def test_single_lists_bit_exact_full_size(torch, n, ne):
    c = casci.Context(0)
    c.build_strings(ne, ne, n)
    Po, Qo, Jo, So = oracle.single_list_c(n, ne)
    for spin in (0, 1):
        P, Q, J, S = c.single_list(spin)
        assert np.array_equal(P, Po) and np.array_equal(Q, Qo)
        assert np.array_equal(J, Jo) and np.array_equal(S, So)


def test_same_spin_operator_rows_n16(torch):
    n, ne = 16, 8
    c, h, eri = make(n, ne, ne, 4)
    col, val = c.same_spin_operator(0)
    N = col.shape[0]
    rng = np.random.default_rng(16)
    rows = np.unique(np.concatenate([[0, 1, N // 2, N - 2, N - 1], rng.integers(0, N, 60)]))
    ref = oracle.h_rows(h, eri, ne, 0, rows)  # (8, 0) system: address = alpha string
    scale = max(np.abs(v).max() for _, v in ref)
    for r, (rc, rv) in zip(rows, ref):
        assert np.array_equal(col[r], rc), r
        assert np.abs(val[r] - rv).max() < 1e-13 * scale, r


def symmetric_vector(torch, Na, parity, seed):
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn(Na, Na, dtype=torch.float64, device="cuda", generator=g)
    C = X + parity * X.t()
    return (C / C.norm()).contiguous()


@pytest.mark.parametrize("n", [4, 6, 8, 10])
@pytest.mark.parametrize("parity", [1, -1])
def test_sigma_parity_path_vs_oracle(torch, n, parity):
    ne = n // 2
    c, h, eri = make(n, ne, ne, 500 + n)
    Na = c.dims["Na"]
    C = symmetric_vector(torch, Na, parity, 7 + n)
    Ch = C.cpu().numpy()
    ref = oracle.sigma(h, eri, ne, ne, Ch)
    scale = max(1.0, np.abs(ref).max())
    gen = c.sigma(C).cpu().numpy()  # the general path (two gathers) on the same vector
    assert np.abs(gen - ref).max() < 1e-12 * scale
    for prec, tol in TOL.items():
        got = c.sigma_parity(C, parity, ab_prec=prec).cpu().numpy()
        assert np.abs(got - ref).max() < tol * scale, prec
        if prec != "f64":
            assert np.abs(got - ref).max() > 1e-14 * scale  # really the low-precision arithmetic


@pytest.mark.parametrize("parity", [1, -1])
def test_sigma_parity_path_full_size_cas16(torch, parity):
    """CAS(16e,16o), 165,636,900 determinants: the one-gather parity path in
    FP64, FP32 and BF16 alpha-beta arithmetic (the builds of the timed
    solver) on sampled rows, and bitwise reproducibility of each."""
    n, ne = 16, 8
    c, h, eri = make(n, ne, ne, 4)
    d = c.dims
    Na, Nd = d["Na"], d["Ndet"]
    C = symmetric_vector(torch, Na, parity, 21)
    rng = np.random.default_rng(33)
    # rows at the edges of the 32-row tiles of the combination pass, the
    # first and last rows and columns, and random determinants
    edges = []
    for ia in (0, 31, 32, 63, 64, Na // 2 - (Na // 2) % 32, Na - 33, Na - 32, Na - 1):
        for ib in (0, 31, 32, Na - 1, int(rng.integers(0, Na))):
            edges.append(ia * Na + ib)
    pick = np.unique(np.concatenate([[0, Nd - 1], edges, rng.integers(0, Nd, 120)]))
    ref = oracle.sigma_rows(h, eri, ne, ne, C.cpu().numpy(), pick)
    scale = max(1.0, np.abs(ref).max())
    idx = torch.from_numpy(pick).cuda()
    for prec, tol in TOL.items():
        S1 = c.sigma_parity(C, parity, ab_prec=prec)
        S2 = c.sigma_parity(C, parity, ab_prec=prec)
        torch.cuda.synchronize()
        assert torch.equal(S1, S2), prec  # bitwise reproducible
        got = S1.view(-1)[idx].cpu().numpy()
        del S1, S2
        assert np.abs(got - ref).max() < tol * scale, prec


def test_zero_eri_ground_state_cas16(torch):
    """Zero two-electron integrals at CAS(16e,16o): the ground state is the sum
    of the 8 lowest orbital energies of h for each spin."""
    n = 16
    h, _, _ = synth.integrals(n, 4)
    eps = np.linalg.eigvalsh(h)
    c = casci.Context(0)
    c.set_integrals(h, np.zeros((n,) * 4))
    c.build_strings(8, 8, n)
    E, _, info = c.davidson(1, 1e-11, vectors=False, r_tol=1e-7)
    assert info["converged"]
    assert abs(E[0] - 2 * eps[:8].sum()) < 1e-10


def test_rotation_invariance_cas12(torch):
    n = 12
    h, eri, _ = synth.integrals(n, 2)
    Q = synth.random_orthogonal(n, 45)
    h2, eri2 = oracle.rotate_integrals(h, eri, Q)
    Es = []
    for hh, ee in ((h, eri), (h2, eri2)):
        c = casci.Context(0)
        c.set_integrals(hh, ee)
        c.build_strings(6, 6, n)
        E, _, info = c.davidson(3, 1e-11, vectors=False, r_tol=1e-7)
        assert info["converged"]
        Es.append(E)
    assert np.abs(Es[0] - Es[1]).max() < 1e-10


def test_spin_square_is_integral_cas12(torch):
    """<S^2> of converged roots at CAS(12,12) (spin ANY) is S(S+1) with integer S."""
    c, h, eri = make(12, 6, 6, 2)
    E, _, info = c.davidson(3, 1e-11, vectors=False, r_tol=1e-7)
    assert info["converged"]
    for s2 in info["s2"]:
        S = 0.5 * (math.sqrt(1.0 + 4.0 * s2) - 1.0)
        assert abs(S - round(S)) < 1e-6, s2
