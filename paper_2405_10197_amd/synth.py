"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This module holds no arithmetic of the method itself: it only draws the
active-space integrals and CI vectors that both sides are fed.

Integral recipe (one active space of ``norb`` orbitals, no point-group
symmetry), drawn with ``numpy.random.default_rng(seed)`` in this order:

1. diagonal of h: ``norb`` draws U[-2, 1] Eh, sorted ascending (orbital 0 is
   the lowest, so string 0 is the aufbau string);
2. off-diagonal h: one N(0, 0.05) draw per upper-triangle pair p < q in
   row-major order, mirrored to keep h symmetric;
3. Cholesky vectors L[P, p, q], P < naux = 3*norb: one N(0, 0.1) draw per
   (P, p <= q) in P-major, row-major order, mirrored in pq;
4. (pq|rs) = sum_P L[P,p,q] L[P,r,s] (chemists' notation). This has the
   8-fold permutational symmetry and is positive semidefinite as an
   (pq)x(rs) matrix, the factorised form of the integral classes in
   Sec. III.B of the paper.

The scalar core energy is 0 for every synthetic workload except the dressed
one below.

Dressed integrals (``dressed_integrals``; the model-space Hamiltonian of a
reference relaxation, Sec. II.C: a similarity-transformed Hamiltonian keeps
the symmetry of a Hermitian operator, (pq|rs) = (qp|sr) = (rs|pq), but not
(pq|rs) = (qp|rs)): the integrals above for ``seed``, then from
``default_rng(seed + 1_000_003)`` in this order: a symmetric N(0, ``amp``)
change of h (upper triangle with the diagonal, row-major, mirrored), a
N(0, ``amp``) tensor X averaged over the four index maps of that symmetry,
(X + X^(qpsr) + X^(rspq) + X^(srqp)) / 4, added to (pq|rs), and a scalar
N(-1, 0.1).
"""
from __future__ import annotations

import numpy as np


def integrals(norb: int, seed: int, naux: int | None = None):
    """Return (h[n,n], eri[n,n,n,n], e_core) as float64 arrays (see module doc)."""
    n = int(norb)
    if n < 1:
        raise ValueError("norb must be >= 1")
    rng = np.random.default_rng(seed)
    h = np.zeros((n, n))
    h[np.arange(n), np.arange(n)] = np.sort(rng.uniform(-2.0, 1.0, size=n))
    iu = np.triu_indices(n, 1)
    off = rng.normal(0.0, 0.05, size=iu[0].size)
    h[iu] = off
    h[(iu[1], iu[0])] = off
    naux = 3 * n if naux is None else int(naux)
    ip = np.triu_indices(n)
    vals = rng.normal(0.0, 0.1, size=(naux, ip[0].size))
    L = np.zeros((naux, n, n))
    L[:, ip[0], ip[1]] = vals
    L[:, ip[1], ip[0]] = vals
    Lm = L.reshape(naux, n * n)
    eri = (Lm.T @ Lm).reshape(n, n, n, n)
    # The BLAS product is symmetric only up to rounding; make the 8-fold
    # symmetry exact (each averaging step preserves the previous ones).
    eri = 0.5 * (eri + eri.transpose(1, 0, 2, 3))
    eri = 0.5 * (eri + eri.transpose(0, 1, 3, 2))
    eri = 0.5 * (eri + eri.transpose(2, 3, 0, 1))
    return np.ascontiguousarray(h), np.ascontiguousarray(eri), 0.0


def dressed_integrals(norb: int, seed: int, amp: float = 0.02):
    """Return (h, eri, e_core) with the 4-fold symmetry only (see module doc)."""
    h, eri, _ = integrals(norb, seed)
    n = h.shape[0]
    rng = np.random.default_rng(seed + 1_000_003)
    iu = np.triu_indices(n)
    dh = np.zeros((n, n))
    dh[iu] = rng.normal(0.0, amp, size=iu[0].size)
    dh[(iu[1], iu[0])] = dh[iu]
    X = rng.normal(0.0, amp, size=(n, n, n, n))
    dv = 0.25 * (X + X.transpose(1, 0, 3, 2) + X.transpose(2, 3, 0, 1) + X.transpose(3, 2, 1, 0))
    e_core = float(rng.normal(-1.0, 0.1))
    return np.ascontiguousarray(h + dh), np.ascontiguousarray(eri + dv), e_core


def ci_vector(n_alpha_strings: int, n_beta_strings: int, seed: int, nvec: int = 1):
    """Seeded N(0,1) CI coefficients, each vector normalised, shape [nvec, Na, Nb]."""
    rng = np.random.default_rng(seed)
    c = rng.normal(0.0, 1.0, size=(nvec, n_alpha_strings, n_beta_strings))
    c /= np.sqrt(np.einsum("kab,kab->k", c, c))[:, None, None]
    return c


def random_orthogonal(n: int, seed: int):
    """Haar-distributed real orthogonal matrix (QR of N(0,1) with R's diagonal made positive)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(size=(n, n))
    q, r = np.linalg.qr(a)
    return q * np.sign(np.diag(r))[None, :]


def batch_sizes(count: int = 64, seed: int = 3, lo: int = 8, hi: int = 10):
    """Active-space sizes for the batched workload: n drawn uniformly from {lo..hi}."""
    rng = np.random.default_rng(seed)
    return [int(x) for x in rng.integers(lo, hi + 1, size=count)]
