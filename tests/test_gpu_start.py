"""Lowest diagonal elements H_II (eq. (hamiltonian)), the determinants the
Davidson start space is built from, selected on the device (histogram of the
diagonal, then the lowest bins sorted on the host) against a full sort of the
diagonal: ascending by value, ties by lower address."""
import numpy as np
import pytest

from paper_2405_10197_amd import casci, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def full_sort(d, want):
    return np.lexsort((np.arange(d.size), d))[:want]


@pytest.mark.parametrize("n,na,nb,seed,ties", [(8, 4, 4, 900, False), (10, 5, 4, 901, False),
                                               (12, 6, 6, 902, False), (10, 5, 5, 903, True)])
def test_lowest_diagonal_matches_full_sort(torch, n, na, nb, seed, ties):
    h, eri, _ = synth.integrals(n, seed)
    if ties:
        # no two-electron part and orbital energies on a coarse grid: many equal
        # diagonal elements, so ties decide the order
        eri = np.zeros_like(eri)
        h = np.diag(np.round(np.diag(h), 1))
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(na, nb, n)
    d = c.diagonal().reshape(-1)
    if ties:
        assert np.unique(d).size < d.size // 10
    for want in sorted({1, 7, 480, min(d.size, 2000), d.size}):
        assert np.array_equal(c.lowest_diagonal(want), full_sort(d, want)), want


def test_lowest_diagonal_all_equal_takes_the_full_selection(torch):
    """A diagonal whose lowest bins hold more than 2^22 entries (here every
    element is equal: no integrals) is selected in full on the host: the
    lowest addresses come first."""
    n, ne = 14, 7
    c = casci.Context(0)
    c.set_integrals(np.zeros((n, n)), np.zeros((n, n, n, n)))
    c.build_strings(ne, ne, n)
    assert c.dims["Ndet"] > (1 << 22)
    assert np.array_equal(c.lowest_diagonal(480), np.arange(480))


def test_lowest_diagonal_argument_checks(torch):
    c = casci.Context(0)
    h, eri, _ = synth.integrals(6, 904)
    c.set_integrals(h, eri)
    c.build_strings(3, 3, 6)
    with pytest.raises(casci.CasciError):
        c.lowest_diagonal(c.dims["Ndet"] + 1)
    assert c.lowest_diagonal(0).size == 0


def test_block_cache_reuses_the_basis_of_a_previous_solve(torch):
    """Two identical solves in one process: the second takes its basis blocks
    from the library's cache (the first left them there) and gives bitwise
    the same energies and iterations; releasing the cache empties it."""
    h, eri, _ = synth.integrals(12, 905)
    out = []
    for rep in range(2):
        c = casci.Context(0)
        c.set_integrals(h, eri)
        c.build_strings(6, 6, 12)
        E, _, info = c.davidson(2, 1e-9, r_tol=1e-5, precond="olsen", vectors=False, history=400, max_iter=400)
        assert info["converged"]
        out.append((E, info["iterations"], info["hist_energy"]))
        del c
        # the basis B and its sigma vectors S (tens of vectors of 6.8 MB each)
        # are kept
        assert casci.cached_bytes(0) >= 2 * (64 << 20)
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert np.array_equal(out[0][2], out[1][2])
    casci.release_cache()
    assert casci.cached_bytes() == 0
