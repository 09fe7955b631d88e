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

The scalar core energy is 0 for every synthetic workload.
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
