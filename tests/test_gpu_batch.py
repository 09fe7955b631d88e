"""Many small active spaces: graph-replayed sigma builds, the gather
autotuner, and concurrent batched solves against single solves and the
oracle."""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

import oracle
from paper_2405_10197_amd import casci, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def electrons(n):
    """CAS(n e, n o): nalpha = ceil(n/2), nbeta = floor(n/2)."""
    return (n + 1) // 2, n // 2


def make(n, seed, own_stream=False):
    na, nb = electrons(n)
    h, eri, _ = synth.integrals(n, seed)
    c = casci.Context(0, own_stream=own_stream)
    c.set_integrals(h, eri)
    c.build_strings(na, nb, n)
    return c, h, eri


def lowest(h, eri, n, k):
    na, nb = electrons(n)
    H = oracle.hamiltonian_csr(h, eri, na, nb)
    return np.sort(sla.eigsh(H, k=k, which="SA", tol=1e-12)[0])


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_graph_replay_reproduces_eager_solve(torch, prec):
    """Every sigma replayed from the captured graph equals the eager build
    bitwise (all reductions have a fixed order), so the whole solve, with eager
    work and synchronisations between the replays, takes exactly the same path:
    the same iterations and bitwise the same energies at every iteration."""
    c, h, eri = make(8, 3000)
    E0, _, i0 = c.davidson(4, 1e-11, r_tol=1e-7, vectors=False, ab_prec=prec, history=500)
    E1, _, i1 = c.davidson(4, 1e-11, r_tol=1e-7, vectors=False, ab_prec=prec, history=500, graph=True)
    assert i0["converged"] and i1["converged"]
    assert i0["iterations"] == i1["iterations"]
    assert np.array_equal(i0["hist_energy"], i1["hist_energy"])
    assert np.array_equal(E0, E1)


WIDTHS = (16, 32, 64, 128, 1602, 3202, 1604, 3204, 6404, 99)


@pytest.mark.parametrize("n", [8, 9])
def test_every_gather_width_matches_oracle(torch, n):
    """Each strip width the autotuner can pick (16/32/64 lanes per entry, or
    64 lanes x 2 columns) gives sigma = H C (FP64 and FP32-input gathers; the
    n = 9 doublet has an odd row length), and the autotuner's choice is one
    of them."""
    c, h, eri = make(n, 3010 + n)
    na, nb = electrons(n)
    d = c.dims
    x = synth.ci_vector(d["Na"], d["Nb"], 5)[0]
    ref = oracle.sigma(h, eri, na, nb, x)
    xt = torch.from_numpy(x).cuda()
    first64 = first32 = None
    for lpe in WIDTHS:
        c.set_tuning(lpe, lpe)
        s64 = c.sigma(xt).cpu().numpy()
        assert np.abs(s64 - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
        s32 = c.sigma(xt, ab_prec="f32").cpu().numpy()
        assert np.abs(s32 - ref).max() < 1e-5 * np.abs(ref).max()
        # the same summation order for every width: bitwise the same results
        first64 = s64 if first64 is None else first64
        first32 = s32 if first32 is None else first32
        assert np.array_equal(s64, first64) and np.array_equal(s32, first32), lpe
    c.set_tuning(0, 0)
    c.sigma(xt)
    c.sigma(xt, ab_prec="f32")
    t = c.tuning()
    assert t["f64"] in WIDTHS and t["f32in"] in WIDTHS


def test_fp32_storage_build_tunes_its_gather(torch):
    """The FP32-storage build (FP32 C and sigma) times its own FP32-output
    gather on the whole space when no width is tuned yet: the choice is one
    of its candidates and sigma matches the oracle to the FP32 bound."""
    c, h, eri = make(10, 3040)
    na, nb = electrons(10)
    d = c.dims
    x = synth.ci_vector(d["Na"], d["Nb"], 8)[0].astype(np.float32)
    ref = oracle.sigma(h, eri, na, nb, x.astype(np.float64))
    s = c.sigma(torch.from_numpy(x).cuda(), ab_prec="f32").cpu().numpy()
    assert c.tuning()["f32in"] in (64, 128, 1604, 3204, 6404, 99)
    assert np.abs(s - ref).max() < 1e-5 * np.abs(ref).max()


def test_bf16_blocked_gather_sums_in_fp32(torch):
    """In a BF16 build the row-blocked gather (width 99) sums in FP32 and the
    other widths in FP64: the two sigmas differ at the FP32 rounding level,
    far inside the BF16 error bound against the oracle."""
    c, h, eri = make(10, 3020)
    na, nb = electrons(10)
    d = c.dims
    x = synth.ci_vector(d["Na"], d["Nb"], 6)[0]
    ref = oracle.sigma(h, eri, na, nb, x)
    xt = torch.from_numpy(x).cuda()
    c.set_tuning(0, 64)
    s64 = c.sigma(xt, ab_prec="bf16").cpu().numpy()
    c.set_tuning(0, 99)
    s99 = c.sigma(xt, ab_prec="bf16").cpu().numpy()
    c.set_tuning(0, 0)
    scale = np.abs(ref).max()
    assert np.abs(s99 - s64).max() < 1e-5 * scale
    assert np.abs(s99 - ref).max() < 2e-2 * scale


@pytest.mark.parametrize("n,dressed", [(10, False), (8, True)])
def test_every_fp64_ab_layout_gives_the_same_bits(torch, n, dressed):
    """FP64 alpha-beta layouts (M tiles per wave x sigma-row chunks in LDS):
    every layout with a kernel variant for the shape gives bitwise the same
    sigma (fixed-point sums), equal to the oracle's; one without a variant is
    refused with an error; the autotuner picks one of those that run."""
    na, nb = electrons(n)
    if dressed:
        h, eri, ec = synth.dressed_integrals(n, 3030 + n)
    else:
        (h, eri, _), ec = synth.integrals(n, 3030 + n), 0.0
    c = casci.Context(0)
    c.set_integrals(h, eri, ec)
    c.build_strings(na, nb, n)
    pairs = 1 if dressed else 0
    d = c.dims
    x = synth.ci_vector(d["Na"], d["Nb"], 7)[0]
    ref = oracle.sigma(h, eri, na, nb, x, ecore=ec)
    xt = torch.from_numpy(x).cuda()
    first, ran = None, []
    for code in (11, 21, 12, 22, 13, 14, 24):
        c.set_ab_layout(pairs, code)
        try:
            s = c.sigma(xt).cpu().numpy()
        except casci.CasciError:
            continue
        ran.append(code)
        first = s if first is None else first
        assert np.array_equal(s, first), code
    assert len(ran) >= 4, ran
    assert np.abs(first - ref).max() < 1e-12 * max(1.0, np.abs(ref).max())
    c.set_ab_layout(pairs, 0)
    assert np.array_equal(c.sigma(xt).cpu().numpy(), first)
    assert c.ab_layout()["full" if dressed else "sym"] in ran


def test_batch_matches_single_solves_and_oracle(torch):
    """Uneven active spaces CAS(8,8) .. CAS(10,10) (CAS(9,9) as a doublet), 4
    roots each, own integrals each, solved concurrently with graph-replayed
    sigma builds: every instance matches its own single solve and (n <= 9) the
    oracle to 1e-10 Eh."""
    ns = [8, 9, 10, 8, 9, 10]
    k = 4
    items = [make(n, 3100 + i, own_stream=True) for i, n in enumerate(ns)]
    E, infos = casci.batch_davidson([c for c, _, _ in items], k, 1e-11, r_tol=1e-7, graph=True, nthreads=6)
    for i, (n, (c, h, eri)) in enumerate(zip(ns, items)):
        assert infos[i]["converged"], (i, n)
        Es, _, _ = c.davidson(k, 1e-11, r_tol=1e-7, vectors=False)
        assert np.abs(E[i] - Es).max() < 1e-10, (i, n, E[i], Es)
        if n <= 9:
            Eo = lowest(h, eri, n, k)
            assert np.abs(E[i] - Eo).max() < 1e-10, (i, n, E[i], Eo)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_batch_mixed_precision_matches_fp64(torch, prec):
    ns = [8, 10, 9, 10]
    k = 4
    items = [make(n, 3200 + i, own_stream=True) for i, n in enumerate(ns)]
    ctxs = [c for c, _, _ in items]
    E64, i64 = casci.batch_davidson(ctxs, k, 1e-11, r_tol=1e-7, graph=True)
    El, il = casci.batch_davidson(ctxs, k, 1e-11, r_tol=1e-7, graph=True, ab_prec=prec, precond="olsen")
    assert all(x["converged"] for x in i64 + il)
    assert np.abs(El - E64).max() < 1e-9
    assert sum(x["sigma_calls_fp64"] for x in il) < sum(x["sigma_calls"] for x in il) / 2
