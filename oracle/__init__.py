"""CPU oracle for string-based CASCI -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. It is a plain, slow, obviously correct
FP64 implementation of what the HIP library computes, and it shares no code
with it:

* the determinant space of Sec. II.A.1 (model-space determinants as
  occupation-number vectors, factorised into alpha and beta strings), with
  strings enumerated by brute force over all 2^n masks and ordered by
  ascending integer value of the mask (bit p = orbital p, Sec. III.C);
* the Hamiltonian of eq. (hamiltonian), as an explicit determinant matrix
  built with the Slater-Condon rules in ``slater_condon.c`` (phases by
  explicit operator application), diagonalised with LAPACK;
* the single-substitution lists of Sec. II.A.1 ("precomputed lists of
  determinants connected by one- and two-electron substitution
  operators"), built by applying a+_p a_q to each string one operator at a
  time;
* S^2 as an explicit matrix, for spin checks (Sec. II.A.1, spin projection);
* one- and two-particle density matrices by operator application.

Pins (tests under ``-m "not gpu"``): brute-force second quantisation of
eq. (hamiltonian) on tiny spaces, the closed-form 2-electron/2-orbital
spectrum, one-electron and (1,1)-electron special cases that reduce to
LAPACK, the zero-ERI spectrum as sums of orbital energies, full occupation,
Hermiticity, integer S(S+1) spectra and invariance of the spectrum under
orthogonal orbital rotations (Sec. II.G).

``mlp_*`` (FP64 forward/backward of the preconditioner network) lives in
``oracle.mlp``.
"""
from __future__ import annotations

import ctypes
import itertools
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "slater_condon.c")
_LIB = os.path.join(_HERE, "liboracle_sc.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile slater_condon.c with gcc into liboracle_sc.so (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        P = ctypes.c_void_p
        lib.oracle_dense_h.argtypes = [i, P, P, d, P, l, P, l, P]
        lib.oracle_sigma_rows.argtypes = [i, P, P, d, P, l, P, l, P, P, l, P]
        lib.oracle_dense_s2.argtypes = [i, P, l, P, l, P]
        lib.oracle_h_rows.argtypes = [i, P, P, d, P, l, P, l, P, l, l, P, P, P]
        lib.oracle_single_list.argtypes = [i, P, l, i, P, P, P, P]
        lib.oracle_rdm.argtypes = [i, P, l, P, l, P, P, P]
        for f in (lib.oracle_dense_h, lib.oracle_sigma_rows, lib.oracle_dense_s2, lib.oracle_h_rows,
                  lib.oracle_single_list, lib.oracle_rdm):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# strings and substitution lists (Sec. II.A.1)
# --------------------------------------------------------------------------
def strings(norb: int, nel: int) -> np.ndarray:
    """All nel-electron strings of norb orbitals, ascending as integers (brute force)."""
    if nel < 0 or nel > norb:
        raise ValueError("need 0 <= nel <= norb")
    if norb <= 20:
        masks = [m for m in range(1 << norb) if bin(m).count("1") == nel]
    else:
        masks = sorted(sum(1 << p for p in c) for c in itertools.combinations(range(norb), nel))
    return np.array(masks, dtype=np.uint64)


def _apply(ops, mask: int):
    """Apply a product of operators, rightmost first. ops: list of ('+'|'-', orbital).
    Returns (sign, mask) or None if the result vanishes."""
    sign = 1
    for kind, p in reversed(ops):
        passed = bin(mask & ((1 << p) - 1)).count("1")
        if kind == "-":
            if not (mask >> p) & 1:
                return None
            mask &= ~(1 << p)
        else:
            if (mask >> p) & 1:
                return None
            mask |= 1 << p
        if passed & 1:
            sign = -sign
    return sign, mask


def single_list(norb: int, nel: int):
    """Single-substitution list of every string I, canonical order.

    For string I the entries are (p, q, J, sign) with <I| a+_p a_q |J> = sign,
    p running over the occupied orbitals of I ascending and, for each p,
    q over (unoccupied orbitals of I) + {p} ascending. J is an address into
    ``strings(norb, nel)``. Returns int arrays p, q, J, sign of shape [N, s].
    """
    strs = [int(x) for x in strings(norb, nel)]
    index = {m: k for k, m in enumerate(strs)}
    P, Q, J, S = [], [], [], []
    for mI in strs:
        pp, qq, jj, ss = [], [], [], []
        occ_ = [p for p in range(norb) if (mI >> p) & 1]
        for p in occ_:
            cands = sorted([q for q in range(norb) if not (mI >> q) & 1] + [p])
            for q in cands:
                # J = the string that a+_p a_q maps onto I: remove p from I, add q
                mJ = (mI & ~(1 << p)) | (1 << q)
                res = _apply([("+", p), ("-", q)], mJ)
                assert res is not None and res[1] == mI
                pp.append(p); qq.append(q); jj.append(index[mJ]); ss.append(res[0])
        P.append(pp); Q.append(qq); J.append(jj); S.append(ss)
    shape = (len(strs), len(P[0]) if P else 0)
    return (np.array(P, dtype=np.int64).reshape(shape), np.array(Q, dtype=np.int64).reshape(shape),
            np.array(J, dtype=np.int64).reshape(shape), np.array(S, dtype=np.int64).reshape(shape))


def single_list_c(norb: int, nel: int):
    """The same single-substitution list as ``single_list`` (same order, same
    operator-by-operator signs), computed in C (``oracle_single_list``) for the
    large string sets (n = 16, 18) that the Python loop would take minutes on."""
    strs = strings(norb, nel)
    N = strs.size
    s = nel * (norb - nel + 1)
    out = [np.empty(N * s, dtype=np.int64) for _ in range(4)]  # J, sign, P, Q
    if N * s:
        rc = _load().oracle_single_list(norb, _ptr(strs), N, s, *(_ptr(a) for a in out))
        if rc != 0:
            raise RuntimeError("oracle_single_list failed: %d" % rc)
    J, S, P, Q = (a.reshape(N, s) for a in out)
    return P, Q, J, S


def h_rows(h, eri, nalpha: int, nbeta: int, rows, ecore: float = 0.0):
    """Rows of the explicit H for the determinant addresses ``rows``: a list of
    (columns ascending, values) per row, from the same Slater-Condon elements
    as ``hamiltonian`` (matrix-free, for spaces too large for a dense H)."""
    n, h, eri = _prep(h, eri)
    a = strings(n, nalpha)
    b = strings(n, nbeta)
    ne = nalpha + nbeta
    maxc = 1 + ne * (2 * n - ne) + math.comb(ne, 2) * math.comb(2 * n - ne, 2)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
    cols = np.empty(rows.size * maxc, dtype=np.int64)
    vals = np.empty(rows.size * maxc)
    cnt = np.empty(rows.size, dtype=np.int64)
    rc = _load().oracle_h_rows(n, _ptr(h), _ptr(eri), float(ecore), _ptr(a), a.size, _ptr(b), b.size,
                               _ptr(rows), rows.size, maxc, _ptr(cols), _ptr(vals), _ptr(cnt))
    if rc != 0:
        raise RuntimeError("oracle_h_rows failed: %d" % rc)
    out = []
    for t in range(rows.size):
        c = cols[t * maxc:t * maxc + cnt[t]]
        v = vals[t * maxc:t * maxc + cnt[t]]
        o = np.argsort(c, kind="stable")
        out.append((c[o], v[o]))
    return out


# --------------------------------------------------------------------------
# Hamiltonian, sigma, S^2 (eq. hamiltonian; Slater-Condon in slater_condon.c)
# --------------------------------------------------------------------------
def _prep(h, eri):
    h = np.ascontiguousarray(h, dtype=np.float64)
    eri = np.ascontiguousarray(eri, dtype=np.float64)
    n = h.shape[0]
    if h.shape != (n, n) or eri.shape != (n, n, n, n):
        raise ValueError("h must be [n,n] and eri [n,n,n,n]")
    return n, h, eri


def hamiltonian(h, eri, nalpha: int, nbeta: int, ecore: float = 0.0) -> np.ndarray:
    """Explicit H over determinants (Ia, Ib) -> Ia*Nb + Ib."""
    n, h, eri = _prep(h, eri)
    a = strings(n, nalpha)
    b = strings(n, nbeta)
    nd = a.size * b.size
    H = np.empty((nd, nd))
    rc = _load().oracle_dense_h(n, _ptr(h), _ptr(eri), float(ecore), _ptr(a), a.size, _ptr(b), b.size, _ptr(H))
    if rc != 0:
        raise RuntimeError("oracle_dense_h failed: %d" % rc)
    return H


def sigma_rows(h, eri, nalpha: int, nbeta: int, C, rows, ecore: float = 0.0) -> np.ndarray:
    """sigma_I = sum_J H_IJ C_J for the determinant addresses in ``rows`` (matrix-free)."""
    n, h, eri = _prep(h, eri)
    a = strings(n, nalpha)
    b = strings(n, nbeta)
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(-1))
    if C.size != a.size * b.size:
        raise ValueError("C has the wrong size")
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64).reshape(-1))
    if rows.size and (rows.min() < 0 or rows.max() >= C.size):
        raise ValueError("row out of range")
    out = np.empty(rows.size)
    rc = _load().oracle_sigma_rows(n, _ptr(h), _ptr(eri), float(ecore), _ptr(a), a.size, _ptr(b), b.size,
                                   _ptr(C), _ptr(rows), rows.size, _ptr(out))
    if rc != 0:
        raise RuntimeError("oracle_sigma_rows failed: %d" % rc)
    return out


def sigma(h, eri, nalpha: int, nbeta: int, C, ecore: float = 0.0) -> np.ndarray:
    """Full sigma = H C (matrix-free), returned with C's [Na, Nb] shape."""
    n = np.asarray(h).shape[0]
    na, nb = strings(n, nalpha).size, strings(n, nbeta).size
    out = sigma_rows(h, eri, nalpha, nbeta, C, np.arange(na * nb), ecore)
    return out.reshape(na, nb)


def hamiltonian_csr(h, eri, nalpha: int, nbeta: int, ecore: float = 0.0, block: int = 4096):
    """H as a scipy CSR matrix (same Slater-Condon elements as ``hamiltonian``),
    for spaces too large for the dense matrix."""
    import scipy.sparse as sp
    n, h, eri = _prep(h, eri)
    a = strings(n, nalpha)
    b = strings(n, nbeta)
    nd = a.size * b.size
    ne = nalpha + nbeta
    maxc = 1 + ne * (2 * n - ne) + math.comb(ne, 2) * math.comb(2 * n - ne, 2)
    L = _load()
    indptr = [0]
    cols_all, vals_all = [], []
    for r0 in range(0, nd, block):
        rows = np.arange(r0, min(nd, r0 + block), dtype=np.int64)
        cols = np.empty(rows.size * maxc, dtype=np.int64)
        vals = np.empty(rows.size * maxc)
        cnt = np.empty(rows.size, dtype=np.int64)
        rc = L.oracle_h_rows(n, _ptr(h), _ptr(eri), float(ecore), _ptr(a), a.size, _ptr(b), b.size,
                             _ptr(rows), rows.size, maxc, _ptr(cols), _ptr(vals), _ptr(cnt))
        if rc != 0:
            raise RuntimeError("oracle_h_rows failed: %d" % rc)
        for t in range(rows.size):
            cols_all.append(cols[t * maxc:t * maxc + cnt[t]])
            vals_all.append(vals[t * maxc:t * maxc + cnt[t]])
        indptr.extend((indptr[-1] + np.cumsum(cnt)).tolist())
    H = sp.csr_matrix((np.concatenate(vals_all), np.concatenate(cols_all), np.array(indptr)), shape=(nd, nd))
    H.sort_indices()
    return H


def s2_matrix(norb: int, nalpha: int, nbeta: int) -> np.ndarray:
    a = strings(norb, nalpha)
    b = strings(norb, nbeta)
    nd = a.size * b.size
    S2 = np.empty((nd, nd))
    rc = _load().oracle_dense_s2(norb, _ptr(a), a.size, _ptr(b), b.size, _ptr(S2))
    if rc != 0:
        raise RuntimeError("oracle_dense_s2 failed: %d" % rc)
    return S2


def diagonal(h, eri, nalpha: int, nbeta: int, ecore: float = 0.0) -> np.ndarray:
    """H_II for every determinant (matrix-free: sigma of unit vectors would be wasteful,
    so for small spaces use the dense matrix)."""
    return np.diag(hamiltonian(h, eri, nalpha, nbeta, ecore)).copy()


def same_spin_operator(h, eri, nel: int) -> np.ndarray:
    """H of the (nel alpha, 0 beta) system without the scalar term: the matrix that
    acts on one spin's strings alone."""
    return hamiltonian(h, eri, nel, 0, 0.0)


def solve(h, eri, nalpha: int, nbeta: int, nroots: int = 1, ecore: float = 0.0, spin: str = "any"):
    """Lowest eigenpairs of H (LAPACK dsyevd through numpy.linalg.eigh).

    spin='any': lowest roots of the full determinant space.
    spin='singlet': lowest roots inside the S^2 = 0 eigenspace.
    Returns (E[nroots], X[nroots, Na, Nb], s2[nroots]); each vector's phase is
    fixed so that its largest-magnitude entry (lowest index on ties) is positive.
    """
    n = np.asarray(h).shape[0]
    na, nb = strings(n, nalpha).size, strings(n, nbeta).size
    H = hamiltonian(h, eri, nalpha, nbeta, ecore)
    S2 = s2_matrix(n, nalpha, nbeta)
    if spin == "any":
        E, X = np.linalg.eigh(H)
    elif spin == "singlet":
        w, U = np.linalg.eigh(S2)
        U = U[:, np.abs(w) < 1e-8]
        if U.shape[1] == 0:
            raise ValueError("no singlet in this determinant space")
        E, Y = np.linalg.eigh(U.T @ H @ U)
        X = U @ Y
    else:
        raise ValueError("spin must be 'any' or 'singlet'")
    E = E[:nroots]
    X = X[:, :nroots].T.copy()
    for k in range(X.shape[0]):
        i = int(np.argmax(np.abs(X[k])))
        if X[k, i] < 0:
            X[k] = -X[k]
    s2 = np.einsum("ki,ij,kj->k", X, S2, X)
    return E, X.reshape(-1, na, nb), s2


def rdm(norb: int, nalpha: int, nbeta: int, C, two: bool = True):
    """Spin-resolved density matrices of a real CI vector C [Na, Nb] (Sec. II.A.1),
    by explicit operator application in ``oracle_rdm``:
    g1[s, p, q] = <C| a+_ps a_qs |C> (s = alpha, beta) and
    g2[k, p, q, r, u] = <C| a+_ps a+_rt a_ut a_qs |C> for (s, t) = (a, a), (a, b), (b, b).
    The cost grows as Ndet n^4: tiny spaces only."""
    strs_a = strings(norb, nalpha)
    strs_b = strings(norb, nbeta)
    C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(-1))
    if C.size != strs_a.size * strs_b.size:
        raise ValueError("C has the wrong size")
    n = norb
    g1 = np.zeros((2, n, n))
    g2 = np.zeros((3, n, n, n, n)) if two else None
    rc = _load().oracle_rdm(n, _ptr(strs_a), strs_a.size, _ptr(strs_b), strs_b.size, _ptr(C), _ptr(g1),
                            _ptr(g2) if two else None)
    if rc != 0:
        raise RuntimeError("oracle_rdm failed: %d" % rc)
    return g1, g2


def spin_free_rdm(g1, g2):
    """Spin-summed density matrices: gamma_pq = sum_s g1[s,p,q] and
    Gamma_pqru = sum_st <a+_ps a+_rt a_ut a_qs>; the (beta, alpha) block is the
    (alpha, beta) one with the pairs (pq) and (ru) exchanged."""
    gam = g1[0] + g1[1]
    Gam = g2[0] + g2[2] + g2[1] + g2[1].transpose(2, 3, 0, 1)
    return gam, Gam


def rdm_energy(h, eri, gam, Gam, ecore: float = 0.0):
    """E = V + sum_pq h_pq gamma_pq + 1/2 sum_pqru (pq|ru) Gamma_pqru (chemists' integrals)."""
    return ecore + float(np.einsum("pq,pq->", h, gam)) + 0.5 * float(np.einsum("pqru,pqru->", eri, Gam))


def rotate_integrals(h, eri, Q):
    """Integrals in the rotated orbitals psi'_p = sum_q psi_q Q_qp (Sec. II.G)."""
    h2 = Q.T @ h @ Q
    e2 = np.einsum("abcd,ap,bq,cr,ds->pqrs", eri, Q, Q, Q, Q, optimize=True)
    return h2, e2
