"""The allocation-free sigma entry point (casci_sigma_noalloc) against the
allocating ones (casci_sigma, casci_sigma_parity) through the C ABI: two
calls in a row, the second on a smaller string space, in every arithmetic
and parity; the size limit and the preconditions are refused cleanly."""
import ctypes

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


def make(n, seed):
    h, eri, _ = synth.integrals(n, seed)
    c = casci.Context(0)
    c.set_integrals(h, eri)
    c.build_strings(n // 2, n // 2, n)
    return c


def vector(torch, c, parity, seed):
    Na = c.dims["Na"]
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.randn(Na, Na, dtype=torch.float64, device="cuda", generator=g)
    C = X if parity == 0 else X + parity * X.t()
    return (C / C.norm()).contiguous()


def test_noalloc_sigma_matches_the_allocating_entry_points(torch):
    L = casci.lib()
    # CAS(12,12) first (853,776 determinants: 20 MB of work space in FP64 with
    # parity 0, 26 MB in BF16), then the smaller CAS(10,10) (63,504)
    for n, seed in ((12, 2), (10, 77)):
        c = make(n, seed)
        for prec in ("f64", "f32", "bf16"):
            for parity in (0, 1, -1):
                C = vector(torch, c, parity, 5 + n + parity)
                if parity == 0:
                    ref = c.sigma(C, ab_prec=prec)  # the allocating path; also builds the tables
                else:
                    ref = c.sigma_parity(C, parity, ab_prec=prec)
                out = torch.full_like(C, float("nan"))
                rc = L.casci_sigma_noalloc(c._h, ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           casci.PREC[prec], parity)
                assert rc == casci.OK, c.last_error()
                torch.cuda.synchronize()
                scale = max(1.0, ref.abs().max().item())
                assert (out - ref).abs().max().item() <= 1e-12 * scale, (n, prec, parity)
                # the same kernels in the same order: bitwise equal in fact
                assert torch.equal(out, ref), (n, prec, parity)


def test_noalloc_refuses_what_it_cannot_do(torch):
    L = casci.lib()
    c = make(10, 3)
    C = vector(torch, c, 0, 1)
    out = torch.empty_like(C)
    pc, po = ctypes.c_void_p(C.data_ptr()), ctypes.c_void_p(out.data_ptr())
    # before any allocating sigma call: operators and tables do not exist yet
    assert L.casci_sigma_noalloc(c._h, pc, po, casci.F64, 0) == casci.E_STATE
    c.sigma(C)  # builds the operators and the FP64 tables
    assert L.casci_sigma_noalloc(c._h, pc, po, casci.F64, 0) == casci.OK
    # the BF16 reduction table is built by the first BF16 build only
    assert L.casci_sigma_noalloc(c._h, pc, po, casci.BF16, 0) == casci.E_STATE
    assert L.casci_sigma_noalloc(c._h, pc, po, casci.F64, 3) == casci.E_ARG
    assert L.casci_sigma_noalloc(c._h, pc, pc, casci.F64, 0) == casci.E_ARG
    # CAS(14,14): 11,778,624 determinants need 283 MB, more than the 64 MiB scratch
    big = casci.Context(0)
    h, eri, _ = synth.integrals(14, 4)
    big.set_integrals(h, eri)
    big.build_strings(7, 7, 14)
    assert L.casci_sigma_noalloc(big._h, pc, po, casci.F64, 0) == casci.E_UNSUPPORTED
    assert "static scratch" in big.last_error()
