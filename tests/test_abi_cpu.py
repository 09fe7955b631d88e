"""C ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and validates arguments and call order in a validate-only
context (device = -1) before any device work."""
import ctypes
import math

import numpy as np
import pytest

from paper_2405_10197_amd import casci, synth


@pytest.fixture(scope="module")
def L():
    return casci.lib()


def test_every_header_symbol_is_exported(L):
    names = casci.header_symbols()
    assert "casci_sigma" in names and "casci_davidson" in names
    for n in names:
        assert hasattr(L, n), n


def vctx():
    return casci.Context(device=-1)


def test_create_rejects_bad_device_and_null(L):
    assert L.casci_create(None, 0, None) == casci.E_ARG
    h = ctypes.c_void_p()
    assert L.casci_create(ctypes.byref(h), -7, None) == casci.E_ARG


def test_dims_after_build_strings():
    c = vctx()
    c.build_strings(8, 8, 16)
    d = c.dims
    assert d["Na"] == d["Nb"] == 12870 and d["Ndet"] == 12870 ** 2
    assert d["sa"] == 8 * 9 and d["ra"] == 1 + 64 + 28 * 28
    c.build_strings(5, 4, 9)
    d = c.dims
    assert (d["Na"], d["Nb"], d["sa"], d["sb"]) == (126, 126, 25, 24)
    assert d["ra"] == 1 + 5 * 4 + math.comb(5, 2) * math.comb(4, 2)


@pytest.mark.parametrize("na,nb,n", [(-1, 0, 4), (5, 1, 4), (1, 1, 0), (1, 1, 65)])
def test_build_strings_rejects_bad_sizes(na, nb, n):
    c = vctx()
    with pytest.raises(casci.CasciError) as e:
        c.build_strings(na, nb, n)
    assert e.value.code == casci.E_ARG


def test_predicted_out_of_memory():
    c = vctx()
    with pytest.raises(casci.CasciError) as e:
        c.build_strings(20, 20, 40)
    assert e.value.code == casci.E_NOMEM
    with pytest.raises(casci.CasciError) as e:
        c.build_strings(12, 12, 24)  # 7.3e6^2 determinants: petabytes
    assert e.value.code == casci.E_NOMEM


def test_integral_validation():
    h, eri, _ = synth.integrals(4, 1)
    c = vctx()
    c.set_integrals(h, eri)
    bad = h.copy()
    bad[0, 1] += 1e-3
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(bad, eri)
    assert e.value.code == casci.E_ARG
    bad = eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h, bad)
    assert e.value.code == casci.E_ARG
    bad = eri.copy()
    bad[1, 1, 1, 1] = np.nan
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h, bad)
    assert e.value.code == casci.E_NONFINITE
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h, eri, e_core=float("inf"))
    assert e.value.code == casci.E_NONFINITE


def test_dressed_integrals_accepted_hermiticity_required():
    # (pq|rs) = (qp|sr) = (rs|pq) is enough (dressed integrals); breaking either
    # of those two relations is an error, breaking only (pq|rs) = (qp|rs) is not
    h, eri, ec = synth.dressed_integrals(4, 2)
    c = vctx()
    c.set_integrals(h, eri, e_core=ec)
    bad = eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    bad[1, 0, 3, 2] += 1e-3            # keeps (pq|rs) = (qp|sr), breaks (rs|pq)
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h, bad)
    assert e.value.code == casci.E_ARG
    bad = eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    bad[2, 3, 0, 1] += 1e-3            # keeps (pq|rs) = (rs|pq), breaks (qp|sr)
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h, bad)
    assert e.value.code == casci.E_ARG
    ok = eri.copy()
    for idx in [(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)]:
        ok[idx] += 1e-3                # the whole 4-fold orbit moves together
    c.set_integrals(h, ok)


def test_call_order_and_norb_mismatch():
    h, eri, _ = synth.integrals(4, 1)
    c = vctx()
    C = np.zeros((6, 6))
    with pytest.raises(casci.CasciError) as e:
        c.sigma(C)
    assert e.value.code == casci.E_STATE
    c.build_strings(2, 2, 4)
    with pytest.raises(casci.CasciError) as e:
        c.sigma(C)
    assert e.value.code == casci.E_STATE      # no integrals yet
    h5, eri5, _ = synth.integrals(5, 1)
    with pytest.raises(casci.CasciError) as e:
        c.set_integrals(h5, eri5)
    assert e.value.code == casci.E_STATE
    c.set_integrals(h, eri)
    with pytest.raises(casci.CasciError) as e:
        c.sigma(C)
    assert e.value.code == casci.E_UNSUPPORTED  # validate-only: everything valid, no device
    with pytest.raises(casci.CasciError) as e:
        c.davidson(1, 1e-8)
    assert e.value.code == casci.E_UNSUPPORTED


def test_davidson_argument_checks():
    h, eri, _ = synth.integrals(4, 1)
    c = vctx()
    c.build_strings(2, 1, 4)
    c.set_integrals(h, eri)
    for kw, code in [(dict(nroots=0), casci.E_ARG), (dict(nroots=33), casci.E_ARG),
                     (dict(tol=-1.0), casci.E_ARG), (dict(spin="singlet"), casci.E_ARG)]:
        args = dict(nroots=1, tol=1e-8)
        args.update(kw)
        with pytest.raises(casci.CasciError) as e:
            c.davidson(args.pop("nroots"), args.pop("tol"), **args)
        assert e.value.code == code, kw


def test_sigma_argument_checks(L):
    c = vctx()
    h, eri, _ = synth.integrals(4, 1)
    c.build_strings(2, 2, 4)
    c.set_integrals(h, eri)
    C = np.zeros((6, 6))
    assert L.casci_sigma(c._h, None, C.ctypes.data, 0, 0, 0) == casci.E_ARG
    assert L.casci_sigma(c._h, C.ctypes.data, C.ctypes.data, 0, 0, 0) == casci.E_ARG
    S = np.zeros((6, 6))
    assert L.casci_sigma(c._h, C.ctypes.data, S.ctypes.data, 7, 0, 0) == casci.E_ARG
    assert L.casci_sigma(c._h, C.ctypes.data, S.ctypes.data, 0, 9, 0) == casci.E_ARG
    assert L.casci_sigma(c._h, C.ctypes.data, S.ctypes.data, 0, 0, 5) == casci.E_ARG
    assert b"NULL" in L.casci_last_error(c._h) or L.casci_last_error(c._h)


def test_struct_layout_matches_binding(L):
    """The ctypes mirrors of the option / info structs agree with the library."""
    import ctypes
    lay = (ctypes.c_int64 * 6)()
    assert L.casci_abi_layout(lay, 6) == 0
    assert list(lay) == [ctypes.sizeof(casci.DavidsonOpts), ctypes.sizeof(casci.DavidsonInfo),
                         casci.DavidsonOpts.progress.offset, casci.DavidsonInfo.residual.offset,
                         casci.DavidsonInfo.hist_energy.offset, casci.DavidsonInfo.hist_len.offset]


def test_batch_rejects_duplicate_contexts_and_bad_tuning(L):
    c = casci.Context(-1)
    with pytest.raises(ValueError):
        casci.batch_davidson([c, c], 1, 1e-8)
    import ctypes
    arr = (ctypes.c_void_p * 2)(c._h, c._h)
    E = np.zeros(2)
    assert L.casci_batch_davidson(arr, 2, 1, 1e-8, None, E.ctypes.data, None, 1) == casci.E_ARG
    assert L.casci_batch_davidson(arr, 0, 1, 1e-8, None, E.ctypes.data, None, 1) == casci.OK
    with pytest.raises(casci.CasciError):
        c.set_tuning(24, 0)


def test_block_cache_calls_without_a_device(L):
    """The device-block cache is empty until something is released on a GPU;
    its calls need no device."""
    assert casci.cached_bytes() == 0
    casci.release_cache()
    casci.release_cache(3)
    assert L.casci_cached_bytes(-1) == 0


def test_ab_layout_codes_checked(L):
    """FP64 alpha-beta layout overrides: 0 or 10 MT + split (MT 1..2, split 1..4)
    per pair set, anything else refused; the context reports what was set."""
    c = casci.Context(-1)
    assert c.ab_layout() == {"sym": 0, "full": 0}
    c.set_ab_layout(0, 21)
    c.set_ab_layout(1, 14)
    assert c.ab_layout() == {"sym": 21, "full": 14}
    c.set_ab_layout(0, 0)
    assert c.ab_layout()["sym"] == 0
    for pairs, code in ((2, 11), (-1, 11), (0, 31), (0, 15), (0, 10), (0, 5), (0, -11), (1, 100)):
        with pytest.raises(casci.CasciError):
            c.set_ab_layout(pairs, code)
    assert c.ab_layout() == {"sym": 0, "full": 14}
    assert L.casci_get_ab_layout(None, None) == casci.E_ARG


def _sym_cases():
    rng = np.random.default_rng(11)
    for n in list(range(1, 41)) + [64, 100, 240]:
        B = rng.standard_normal((n, n))
        yield "random", B + B.T
        yield "diagonal", np.diag(rng.standard_normal(n))
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = np.repeat(rng.standard_normal((n + 2) // 3), 3)[:n]
        yield "triples", (Q * ev) @ Q.T
        ev2 = np.sort(rng.standard_normal(n))
        ev2[: n // 2] = ev2[0] + 1e-13 * np.arange(n // 2)
        yield "cluster", (Q * ev2) @ Q.T
        yield "zero", np.zeros((n, n))
        G = B + B.T
        G[(np.arange(n)[:, None] % 2) != (np.arange(n)[None, :] % 2)] = 0.0
        yield "two blocks", G
        yield "graded", np.diag(10.0 ** np.linspace(-8, 8, n)) + 1e-3 * (B + B.T)


def test_sym_eig_matches_lapack():
    """The solver's host eigensolver (Rayleigh-Ritz and start-space blocks)
    against LAPACK: eigenvalues, residuals and orthonormality to a few ulps
    times n, including repeated, clustered, zero and graded spectra."""
    count = 0
    for name, A in _sym_cases():
        n = A.shape[0]
        w, Z = casci.sym_eig(A)
        ref = np.linalg.eigvalsh(A)
        s = max(1.0, float(np.abs(ref).max()))
        assert np.abs(w - ref).max() <= 1e-14 * n * s, (name, n)
        assert np.all(np.diff(w) >= 0), (name, n)
        assert np.abs(A @ Z - Z * w).max() <= 1e-14 * n * s, (name, n)
        assert np.abs(Z.T @ Z - np.eye(n)).max() <= 1e-14 * n, (name, n)
        count += 1
    assert count == 7 * 43


def test_sym_eig_arguments():
    w, Z = casci.sym_eig(np.zeros((0, 0)))
    assert w.shape == (0,) and Z.shape == (0, 0)
    A = np.eye(3)
    A[1, 2] = A[2, 1] = np.nan
    with pytest.raises(casci.CasciError) as e:
        casci.sym_eig(A)
    assert e.value.code == casci.E_NONFINITE
    # only the lower triangle is read
    A = np.array([[2.0, 99.0], [1.0, 2.0]])
    w, _ = casci.sym_eig(A)
    assert np.allclose(w, [1.0, 3.0], rtol=0, atol=1e-15)


# --------------------------------------------------------------------------
# the binding rejects wrong-sized, wrongly typed or misplaced buffers before
# any library call (a wrong size would make the kernels run out of bounds)
# --------------------------------------------------------------------------
def _ctx633():
    h, eri, _ = synth.integrals(6, 1)
    c = vctx()
    c.set_integrals(h, eri)
    c.build_strings(3, 3, 6)
    return c


def test_binding_rejects_bad_vector_arguments():
    c = _ctx633()
    nd = c.dims["Ndet"]
    with pytest.raises(ValueError):
        c.sigma(np.zeros(nd - 1))
    with pytest.raises(TypeError):
        c.sigma(np.zeros(nd, dtype=np.int64))
    with pytest.raises(ValueError):
        c.sigma(np.zeros(nd), out=np.zeros(nd + 1))
    with pytest.raises(ValueError):
        c.sigma(np.zeros(nd), out=np.zeros(nd, dtype=np.float32))
    with pytest.raises(ValueError):
        c.sigma_parity(np.zeros(nd - 3), 1)
    with pytest.raises(TypeError):
        c.sigma_parity(np.zeros(nd, dtype=np.float32), 1)
    with pytest.raises(ValueError):
        c.diagonal(out=np.zeros(nd + 5))
    with pytest.raises(TypeError):
        c.diagonal(out=np.zeros(nd, dtype=np.float32))
    with pytest.raises(ValueError):
        c.spin_square(np.zeros(2 * nd))
    with pytest.raises(ValueError):
        c.davidson(2, 1e-8, guess=np.zeros((2, nd - 1)))
    with pytest.raises(ValueError):
        c.davidson(2, 1e-8, vectors_out=np.zeros((1, nd)))
    with pytest.raises(ValueError):
        c.mlp_train(np.zeros((10, 8), dtype=np.float32), np.zeros(9, dtype=np.float32))
    with pytest.raises(TypeError):
        c.mlp_train(np.zeros((10, 8)), np.zeros(10, dtype=np.float32))


def test_binding_rejects_host_arrays_where_device_tensors_are_needed():
    c = _ctx633()
    nd = c.dims["Ndet"]
    x = np.zeros(nd)
    with pytest.raises(ValueError):
        c.mlp_features(x, x, 0.0, [0, 1])


def test_mlp_features_index_range_checked_in_the_abi(L):
    c = _ctx633()
    nd = c.dims["Ndet"]
    F = np.zeros((2, 8), dtype=np.float32)
    for bad in ([0, nd], [-1, 3]):
        idx = np.array(bad, dtype=np.int64)
        # non-null stand-in pointers: the range check comes before any device work
        rc = L.casci_mlp_features(c._h, ctypes.c_void_p(16), ctypes.c_void_p(16), 0.0, idx.ctypes.data, 2,
                                  F.ctypes.data)
        assert rc == casci.E_ARG
        assert "out of range" in c.last_error()


def test_sigma_parity_argument_checks(L):
    c = _ctx633()
    nd = c.dims["Ndet"]
    C = np.zeros(nd)
    S = np.zeros(nd)
    assert L.casci_sigma_parity(c._h, C.ctypes.data, S.ctypes.data, casci.F64, 0, casci.MEM_HOST) == casci.E_ARG
    assert L.casci_sigma_parity(c._h, C.ctypes.data, S.ctypes.data, casci.F64, 2, casci.MEM_HOST) == casci.E_ARG
    # validate-only: a valid call stops at the device check
    assert L.casci_sigma_parity(c._h, C.ctypes.data, S.ctypes.data, casci.BF16, -1,
                                casci.MEM_HOST) == casci.E_UNSUPPORTED
    h, eri, _ = synth.integrals(5, 2)
    d = vctx()
    d.set_integrals(h, eri)
    d.build_strings(3, 2, 5)
    nd = d.dims["Ndet"]
    C = np.zeros(nd)
    S = np.zeros(nd)
    assert L.casci_sigma_parity(d._h, C.ctypes.data, S.ctypes.data, casci.F64, 1, casci.MEM_HOST) == casci.E_ARG
    assert "nalpha == nbeta" in d.last_error()


def test_rdm_argument_checks(L):
    c = vctx()
    C = np.zeros(16)
    g1 = np.zeros((2, 4, 4))
    # strings first
    assert L.casci_rdm(c._h, C.ctypes.data, casci.MEM_HOST, g1.ctypes.data, None) == casci.E_STATE
    c.build_strings(2, 2, 4)
    C = np.zeros(c.dims["Ndet"])
    assert L.casci_rdm(c._h, None, casci.MEM_HOST, g1.ctypes.data, None) == casci.E_ARG
    assert L.casci_rdm(c._h, C.ctypes.data, 7, g1.ctypes.data, None) == casci.E_ARG
    assert L.casci_rdm(c._h, C.ctypes.data, casci.MEM_HOST, None, None) == casci.E_ARG
    # integrals are not needed; a validate-only context stops at the device check
    assert L.casci_rdm(c._h, C.ctypes.data, casci.MEM_HOST, g1.ctypes.data, None) == casci.E_UNSUPPORTED
    assert L.casci_rdm_spin_free(c._h, C.ctypes.data, casci.MEM_HOST, g1.ctypes.data, None) == casci.E_UNSUPPORTED
    with pytest.raises(ValueError):
        c.rdm(np.zeros(c.dims["Ndet"] + 1))


@pytest.mark.parametrize("nb", [1, 2, 3, 7, 64, 403, 1520])
def test_tile_pairs_enumerate_the_upper_triangle(nb):
    """The closed-form inversion the parity combination pass uses to find its
    tile pair from the workgroup index: every pair bi <= bj < nb exactly once,
    in row-by-row order (nb = 403: CAS(16,16), 1520: CAS(18,18) 32-row tiles)."""
    got = casci.tile_pairs(nb)
    bi, bj = np.triu_indices(nb)
    assert np.array_equal(got[:, 0], bi) and np.array_equal(got[:, 1], bj)


@pytest.mark.parametrize("n", [1, 31, 32, 33, 100, 252])
def test_tile_pairs_write_every_element_once(n):
    """The parity combination writes tile (bi, bj) and, for bi != bj, its mirror
    (bj, bi), 32 x 32 elements each clipped to the n x n matrix: over all pairs
    every element is written exactly once, so the squares summed per pair (the
    norm the Gram-Schmidt reads from that pass) add up to the whole vector's."""
    nb = (n + 31) // 32
    count = np.zeros((n, n), dtype=np.int64)
    for bi, bj in casci.tile_pairs(nb):
        count[bi * 32:(bi + 1) * 32, bj * 32:(bj + 1) * 32] += 1
        if bi != bj:
            count[bj * 32:(bj + 1) * 32, bi * 32:(bi + 1) * 32] += 1
    assert np.all(count == 1)


def test_tile_pairs_range_checks():
    assert casci.tile_pairs(5, 14, 1).tolist() == [[4, 4]]
    for args in [(0, 0, 1), (5, 15, 1), (5, -1, 1), (5, 10, 6)]:
        with pytest.raises(casci.CasciError) as e:
            casci.tile_pairs(*args)
        assert e.value.code == casci.E_ARG
