"""Row-blocked form of a same-spin operator (the tables the row-blocked
alpha-alpha / beta-beta gather reads), built by the library's host code and
checked without a device: a NumPy emulation of the gather that reads only
the tables reproduces the sparse product sigma = F X of the row form it was
built from, every entry appears in exactly one slot, and padded slots carry
zero."""
import itertools

import numpy as np
import pytest

from paper_2405_10197_amd import casci

CH, ROWB = 64, 512


def row_form(n, ne, seed):
    """Same-spin operator structure of n orbitals / ne electrons (strings in
    ascending integer order): per row the diagonal, then every string that
    differs by one or two replacements, ascending; random values."""
    strs = np.array(sorted(sum(1 << p for p in c) for c in itertools.combinations(range(n), ne)), dtype=np.int64)
    N = strs.size
    rows = []
    for i in range(N):
        x = strs ^ strs[i]
        pc = np.array([bin(int(v)).count("1") for v in x])
        nb = np.nonzero((pc > 0) & (pc <= 4))[0]
        rows.append(np.concatenate([[i], nb]))
    r = len(rows[0])
    assert all(len(x) == r for x in rows)
    col = np.array(rows, dtype=np.int32)
    val = np.random.default_rng(seed).standard_normal(col.shape)
    return col, val


def emulate(col, val, R, t, X):
    N, r = col.shape
    Y = val[:, :1] * X  # the diagonal, read from the row itself
    seen = np.zeros(col.shape, dtype=np.int64)
    pos = {(i, int(j)): e for i in range(N) for e, j in enumerate(col[i])}
    for b, (ux, un, gz, nch) in enumerate(t["binfo"]):
        U = t["uni"][ux:ux + un].astype(np.int64)
        assert np.all(np.diff(U) > 0) and un <= nch * CH
        for w in range(R):
            i = b * R + w
            if i >= N:
                continue
            go = t["goff"][gz + w * (nch + 1): gz + (w + 1) * (nch + 1)].astype(np.int64)
            assert go[0] == 0 and np.all(np.diff(go) >= 0)
            base = t["rbase"][i]
            for ch in range(nch):
                for g in range(base + go[ch], base + go[ch + 1]):
                    for k in range(4):
                        off, v = int(t["goffs"][g, k]), t["gvals"][g, k]
                        assert off % ROWB == 0 and off // ROWB < CH
                        j = U[ch * CH + off // ROWB]
                        if v != 0.0:
                            e = pos[(i, int(j))]
                            assert e > 0 and v == val[i, e]
                            seen[i, e] += 1
                        Y[i] += v * X[j]
    assert np.all(seen[:, 1:] == 1) and np.all(seen[:, 0] == 0)
    return Y


@pytest.mark.parametrize("n,ne", [(8, 4), (9, 4), (10, 5)])
@pytest.mark.parametrize("R", [16, 32])
def test_blocked_tables_reproduce_the_sparse_product(n, ne, R):
    col, val = row_form(n, ne, 100 + n + R)
    t = casci.ss_block_tables(col, val, R)
    assert t is not None
    N = col.shape[0]
    assert t["binfo"].shape[0] == (N + R - 1) // R
    X = np.random.default_rng(7).standard_normal((N, 3))
    F = np.zeros((N, N))
    F[np.repeat(np.arange(N), col.shape[1]), col.reshape(-1)] = val.reshape(-1)
    assert np.allclose(emulate(col, val, R, t, X), F @ X, rtol=0, atol=1e-12 * np.abs(F @ X).max())


def test_blocked_tables_reject_bad_rows():
    col, val = row_form(6, 3, 1)
    bad = col.copy()
    bad[3, 2], bad[3, 3] = bad[3, 3], bad[3, 2]  # not ascending
    with pytest.raises(casci.CasciError):
        casci.ss_block_tables(bad, val, 16)
    with pytest.raises(casci.CasciError):
        casci.ss_block_tables(col, val, 24)


def test_fp32_sums_in_the_canonical_order_stay_near_fp32_rounding():
    """The BF16 build's gather sums in FP32 from FP32 values and an FP32 copy
    of C in the canonical order (accumulator k takes the entries e = k mod 4
    of each row in ascending order, the diagonal first into accumulator 0,
    total (a0 + a1) + (a2 + a3)). Emulated on the tables at CAS(10,10)-like
    structure, the result stays within a few units of FP32 rounding of the
    FP64 product, far below the ~1e-3 of the BF16 alpha-beta term."""
    col, val = row_form(10, 5, 321)
    t = casci.ss_block_tables(col, val, 32)
    N, r = col.shape
    X = np.random.default_rng(8).standard_normal((N, 4))
    X32 = X.astype(np.float32)
    v32 = val.astype(np.float32)
    acc = np.zeros((N, 4, X.shape[1]), dtype=np.float32)
    acc[:, 0] = v32[:, :1] * X32
    for b, (ux, un, gz, nch) in enumerate(t["binfo"]):
        U = t["uni"][ux:ux + un].astype(np.int64)
        for w in range(32):
            i = b * 32 + w
            if i >= N:
                continue
            go = t["goff"][gz + w * (nch + 1): gz + (w + 1) * (nch + 1)].astype(np.int64)
            base = t["rbase"][i]
            for ch in range(nch):
                for g in range(base + go[ch], base + go[ch + 1]):
                    for k in range(4):
                        j = U[ch * CH + int(t["goffs"][g, k]) // ROWB]
                        acc[i, k] += np.float32(t["gvals"][g, k]) * X32[j]
    y = (acc[:, 0] + acc[:, 1]) + (acc[:, 2] + acc[:, 3])
    F = np.zeros((N, N))
    F[np.repeat(np.arange(N), r), col.reshape(-1)] = val.reshape(-1)
    ref = F @ X
    rel = np.abs(y.astype(np.float64) - ref).max() / np.abs(ref).max()
    assert 1e-9 < rel < 1e-5, rel
