"""Benchmark of the string-CASCI hot path on one MI355X.

A step is one complete CASCI solve of the workload on seeded synthetic
integrals: integrals in, strings and substitution lists, same-spin
operators, diagonal, then Davidson-Liu with sigma builds to convergence
(energy change 1e-10 Eh, residual 1e-6). `value` is the time until every
root stays within 1e-8 Eh of the reference energies (median over the timed
steps). The reference energies and the baseline time come from the plain
FP64, diagonal-preconditioned Davidson run in the same process, converged to
a residual below 1e-7; the timed steps use the headline solver: BF16
alpha-beta arithmetic (FP32 accumulation) for the sigma of every correction
vector, FP64 sigma of the Ritz vectors at every collapse (48-vector
subspace) and for the convergence check; Olsen preconditioner; one
same-spin gather per sigma through transposition parity.

Order of the run: the CPU oracle on the host cores (bounded, before any GPU
work, so that it does not compete with the GPU solves for the host), the
FP64 reference solve, then warm-up and timed steps while the wall-clock
budget (--budget-s, counted from the start of the process) allows another
step; at least one timed step always runs. The executed and the requested
step counts are both reported. The JSON line is printed as soon as the timed
steps end.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cas16|cas12]
       python bench.py --sigma-only f64|f32|bf16 --steps K   (kernel profiling aid)
       python bench.py --copy-probe GIB                       (counter calibration: one plain copy)
       python bench.py --batch [--batch-count 64]             (64 uneven CAS(8..10) solves, 4 roots)
       python bench.py --cas18                                (CAS(18,18) sigma throughput, FP32 storage)
       python bench.py --mlp                                  (learned preconditioner trained at scale vs Olsen)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "σ-build GB/s & MFMA util; Davidson time-to-1e-8 Eh CAS(16,16) mixed vs FP64"
PEAK = {"hbm_GBps": 8000.0, "f64_TF": 78.6, "f32_TF": 157.3, "bf16_TF": 2500.0}

WORKLOADS = {
    # name: (norb, nalpha, nbeta, nroots, seed, spin, description)
    "cas16": (16, 8, 8, 3, 4, "any", "CAS(16e,16o), 3 roots state-averaged (equal weights), "
              "165,636,900 determinants, seeded synthetic integrals (seed 4)"),
    "dressed14": (14, 7, 7, 3, 4, "any", "CAS(14e,14o) on dressed integrals ((pq|rs) = (qp|sr) = (rs|pq) "
                  "only: the model-space Hamiltonian of a reference relaxation), 3 roots, 11,778,624 "
                  "determinants, seeded synthetic integrals (seed 4)"),
    "dressed16": (16, 8, 8, 3, 4, "any", "CAS(16e,16o) on dressed integrals ((pq|rs) = (qp|sr) = (rs|pq) "
                  "only), 3 roots, 165,636,900 determinants, seeded synthetic integrals (seed 4)"),
    "cas12": (12, 6, 6, 1, 2, "singlet", "CAS(12e,12o) singlet ground state, 853,776 determinants, "
              "seeded synthetic integrals (seed 2)"),
}
HEADLINE = dict(precond="olsen", ab_prec="bf16", m_max=48)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def progress_printer(tag):
    def f(it, th, rn, ms):
        if it % 10 == 0:
            log("[%s] iter %3d  %.1f s  E %s  |r| %s" % (tag, it, ms / 1000.0,
                                                       " ".join("%.10f" % x for x in th),
                                                       " ".join("%.1e" % x for x in rn)))
    return f


def time_to_threshold(hist_e, hist_t, eref, thr=1e-8):
    """Wall time (s) of the first iteration after which every root stays within thr of eref."""
    err = np.abs(hist_e - eref[None, :]).max(axis=1)
    ok = err < thr
    for i in range(len(ok)):
        if ok[i:].all():
            return hist_t[i] / 1000.0, i
    return float("nan"), -1


T_START = time.time()


def parse_traffic(path):
    """HBM bytes per launch from a committed rocprofv3 counter summary: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), each scaled by what the same counter
    reads for a plain copy of known size (fetch_scale, write_scale), or None."""
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    vals = {}
    for key in ("FETCH_SIZE_KiB", "WRITE_SIZE_KiB", "fetch_scale", "write_scale"):
        m = re.search(r"^%s\s*[:=]\s*([0-9.eE+-]+)" % key, txt, re.M)
        if m:
            vals[key] = float(m.group(1))
    if len(vals) < 4:
        return None
    return 1024.0 * (vals["FETCH_SIZE_KiB"] * vals["fetch_scale"] + vals["WRITE_SIZE_KiB"] * vals["write_scale"])


def sources_sha256(names):
    """SHA-256 over the named kernel sources (paths relative to the repository root)."""
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_traffic(path):
    """The counter traffic of a summary if it was taken on the kernel as it is now:
    the summary names the kernel's sources ('kernel_sources:') and their SHA-256
    at measurement time ('kernel_sources_sha256:'); any change since then makes
    the figure stale and this returns None."""
    b = parse_traffic(path)
    if b is None:
        return None
    txt = open(path).read()
    m1 = re.search(r"^kernel_sources\s*:\s*(.+)$", txt, re.M)
    m2 = re.search(r"^kernel_sources_sha256\s*:\s*([0-9a-f]{64})\s*$", txt, re.M)
    if not m1 or not m2:
        return None
    try:
        now = sources_sha256(m1.group(1).split())
    except OSError:
        return None
    return b if now == m2.group(1) else None


def workload_integrals(name, n, seed):
    """(h, eri, e_core) of a workload: dressed (4-fold symmetric) or ordinary integrals."""
    from paper_2405_10197_amd import synth
    if name.startswith("dressed"):
        return synth.dressed_integrals(n, seed)
    return synth.integrals(n, seed)


def make_ctx(casci, h, eri, n, na, nb, e_core=0.0):
    ctx = casci.Context(0)
    ctx.set_integrals(h, eri, e_core)
    ctx.build_strings(na, nb, n)
    return ctx


def sigma_only(args, casci, h, eri, n, na, nb, e_core=0.0):
    """Repeated sigma builds on a seeded normalised vector (for kernel profiling)."""
    import torch
    ctx = make_ctx(casci, h, eri, n, na, nb, e_core)
    d = ctx.dims
    g = torch.Generator(device="cuda").manual_seed(50)
    C = torch.randn(d["Na"], d["Nb"], dtype=torch.float64, device="cuda", generator=g)
    C /= C.norm()
    S = torch.empty_like(C)
    for _ in range(args.warmup):
        ctx.sigma(C, out=S, ab_prec=args.sigma_only)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        ctx.sigma(C, out=S, ab_prec=args.sigma_only)
        torch.cuda.synchronize()
        log("[sigma] build %d done" % i)
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    P = ctx.profile_read()
    k = max(P["sigma_builds"], 1)
    print(json.dumps({"sigma_only": args.sigma_only, "workload": args.workload, "ms_per_sigma": dt * 1e3,
                      "parts_ms": {x: P[x] / k for x in ("aa_ms", "bb_ms", "ab_ms", "combine_ms", "total_ms")}}))


def batch_mode(args):
    """64 independent solves, CAS(n,n) with n drawn uniformly from {8, 9, 10}
    (seeded), integrals seed 3000 + i, 4 roots each, spin ANY: concurrent
    batched solves (graph-replayed sigma) in FP64, FP32 and BF16 alpha-beta
    arithmetic, against the same solves run one after another."""
    import torch
    from paper_2405_10197_amd import casci, synth
    rng = np.random.default_rng(3)
    ns = rng.integers(8, 11, args.batch_count)
    k = 4
    def contexts():
        out = []
        for i, n in enumerate(ns):
            h, eri, _ = synth.integrals(int(n), 3000 + i)
            c = casci.Context(0, own_stream=True)
            c.set_integrals(h, eri)
            c.build_strings((int(n) + 1) // 2, int(n) // 2, int(n))
            out.append(c)
        return out
    res = {}
    ref = None
    for prec in ("f64", "f32", "bf16"):
        ctxs = contexts()
        kw = dict(r_tol=1e-7, graph=True, ab_prec=prec, precond="olsen" if prec != "f64" else "diag")
        casci.batch_davidson(ctxs[:4], k, 1e-11, **kw)  # warm-up: kernels loaded, autotuner filled
        ctxs = contexts()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E, infos = casci.batch_davidson(ctxs, k, 1e-11, **kw)
        dt = time.perf_counter() - t0
        log("[batch] %s: %.2f s for %d solves" % (prec, dt, len(ctxs)))
        if ref is None:
            ref = E
        res[prec] = {"seconds": dt, "solves_per_s": len(ctxs) / dt, "converged": sum(x["converged"] for x in infos),
                     "max_energy_error_vs_fp64": float(np.abs(E - ref).max()),
                     "sigma_calls": sum(x["sigma_calls"] for x in infos),
                     "sigma_calls_fp64": sum(x["sigma_calls_fp64"] for x in infos)}
    ctxs = contexts()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in ctxs:
        c.davidson(k, 1e-11, r_tol=1e-7, vectors=False)
    seq = time.perf_counter() - t0
    log("[batch] sequential FP64: %.2f s" % seq)
    print(json.dumps({"metric": "batched uneven CASCI solves", "value": res["bf16"]["solves_per_s"],
                      "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "bf16+f64",
                      "data": "synthetic",
                      "config": {"workload": "%d instances CAS(8..10), 4 roots, spin any" % len(ns),
                                 "sizes": {str(n): int((ns == n).sum()) for n in (8, 9, 10)}},
                      "batched": res, "sequential_fp64_seconds": seq}))


def cas18_mode(args):
    """Single sigma(C) calls at CAS(18e,18o) (2,363,904,400 determinants) on
    a seeded normalised random C (N(0,1) from seed 50, drawn in FP64 and
    normalised, then rounded to FP32 storage): FP32-storage builds with FP32
    and BF16 alpha-beta arithmetic, against the FP64 build of the same rounded
    values upcast."""
    import torch
    from paper_2405_10197_amd import casci, synth
    n = args.cas18_norb
    ne = n // 2
    h, eri, _ = synth.integrals(n, 5)
    ctx = casci.Context(0)
    t0 = time.perf_counter()
    ctx.set_integrals(h, eri)
    ctx.build_strings(ne, ne, n)
    d = ctx.dims
    Na, Nb, Nd = d["Na"], d["Nb"], d["Ndet"]
    g = torch.Generator(device="cuda").manual_seed(50)
    C = torch.empty((Na, Nb), dtype=torch.float32, device="cuda")
    rows = max(1, (1 << 27) // Nb)
    for r0 in range(0, Na, rows):  # drawn in FP64 slab by slab, rounded to FP32
        C[r0:r0 + rows] = torch.randn((min(rows, Na - r0), Nb), dtype=torch.float64, device="cuda",
                                      generator=g).to(torch.float32)
    nrm = float(torch.linalg.vector_norm(C.view(-1), dtype=torch.float64))
    C /= nrm
    S = torch.empty_like(C)
    log("[cas18] %d determinants, vectors %.1f GB each in FP32; setup %.1f s" % (Nd, Nd * 4 / 1e9,
                                                                                   time.perf_counter() - t0))
    M = n * (n + 1) // 2
    ab_flops = 2.0 * M * d["sa"] * Nd
    out = {}
    results = {}
    for prec in ("f32", "bf16"):
        ctx.sigma(C, out=S, ab_prec=prec)  # first build: tables, autotuner
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.sigma(C, out=S, ab_prec=prec)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        P = ctx.profile_read()["lowp"]
        ctx.profile(False)
        k = max(P["sigma_builds"], 1)
        aa, bb, ab = P["aa_ms"] / k, P["bb_ms"] / k, P["ab_ms"] / k
        gather_bytes = Nd * 4.0 * 2 + Na * d["ra"] * 12.0
        out[prec] = {"ms_per_sigma": dt * 1e3, "alpha_alpha_ms": aa, "beta_beta_ms": bb, "alpha_beta_ms": ab,
                     "gather_GBps_algorithmic": gather_bytes / (aa * 1e-3) / 1e9,
                     "gather_GBps_gathered_operands": d["ra"] * Nd * 4.0 / (aa * 1e-3) / 1e9,
                     "alpha_beta_TFLOPs": ab_flops / (ab * 1e-3) / 1e12,
                     "alpha_beta_mfma_util": ab_flops / (ab * 1e-3) / 1e12 / (PEAK["f32_TF"] if prec == "f32" else PEAK["bf16_TF"])}
        results[prec] = S.clone() if prec == "f32" else S
        log("[cas18] %s: %.0f ms per sigma (aa %.0f, bb %.0f, ab %.0f)" % (prec, dt * 1e3, aa, bb, ab))
    # FP64 reference of the same rounded values
    s32 = results.pop("f32")
    s16 = results.pop("bf16")
    del S
    torch.cuda.empty_cache()
    C64 = C.to(torch.float64)
    S64 = torch.empty_like(C64)
    t0 = time.perf_counter()
    ctx.sigma(C64, out=S64, ab_prec="f64")
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    nref = float(torch.linalg.vector_norm(S64.view(-1)))
    for prec, sv in (("f32", s32), ("bf16", s16)):
        diff = 0.0
        for r0 in range(0, Na, rows):
            diff += float(((sv[r0:r0 + rows].to(torch.float64) - S64[r0:r0 + rows]) ** 2).sum())
        out[prec]["rel_error_vs_fp64"] = math.sqrt(diff) / nref
    log("[cas18] FP64 reference sigma %.1f s" % t64)
    print(json.dumps({"metric": "CAS(18,18) sigma build, FP32 storage", "value": out["bf16"]["ms_per_sigma"],
                      "unit": "ms per sigma", "n_gpus": 1, "higher_is_better": False, "dtype": "f32 storage",
                      "data": "synthetic", "config": {"workload": "CAS(%de,%do), %d determinants, integrals seed 5, "
                                                                   "C seed 50" % (n, n, Nd)},
                      "sigma": out, "fp64_reference_seconds": t64,
                      "alpha_beta_flops": ab_flops}))


def mlp_init(seed):
    """Scaled Gaussian start of the 8 -> 64 -> 64 -> 1 network (std 1/sqrt(fan_in), zero biases),
    in the parameter layout of the library (W1[8][64], b1, W2[64][64], b2, W3[64], b3)."""
    rng = np.random.default_rng(seed)
    W1 = rng.normal(0, 1 / math.sqrt(8), (8, 64))
    W2 = rng.normal(0, 1 / math.sqrt(64), (64, 64))
    W3 = rng.normal(0, 1 / math.sqrt(64), 64)
    return np.concatenate([W1.ravel(), np.zeros(64), W2.ravel(), np.zeros(64), W3, [0.0]]).astype(np.float32)


def mlp_mode(args):
    """The learned preconditioner at its configured scale: residual -> converged-
    correction pairs from the solver's own iterations (FP64 sigma, Olsen, 3 roots)
    on CAS(12,12) seeds 4100-4107 and CAS(14,14) seeds 4200-4203, the validation
    loss on the held-out CAS(14,14) seed 4204, training on the GPU with the
    library's kernels, then iterations on the held-out CAS(14,14) and the
    CAS(16,16) workload (seed 4, the headline's mixed-precision sigma) with the
    learned preconditioner against Olsen. The energies both solves reach are
    compared; the time-to-1e-8 Eh of each is taken against the Olsen solve's
    converged energies. The result is reported whatever its sign."""
    import torch
    from paper_2405_10197_amd import casci, synth
    k = 3
    t_start = time.perf_counter()

    def context(n, seed):
        h, eri, _ = synth.integrals(n, seed)
        c = casci.Context(0)
        c.set_integrals(h, eri)
        c.build_strings(n // 2, n // 2, n)
        return c

    def collect(n, seed, samples):
        c = context(n, seed)
        d = c.dims
        xs = torch.empty((k, d["Na"], d["Nb"]), dtype=torch.float64, device="cuda")
        _, _, info = c.davidson(k, 1e-12, precond="olsen", r_tol=1e-8, vectors_out=xs, max_iter=2000)
        F, T = c.mlp_collect(k, 1e-10, xs, samples=samples, seed=seed, precond="olsen", max_rows=1 << 22,
                             max_iter=2000)
        log("[mlp] CAS(%d,%d) seed %d: %d iterations to the converged vectors, %d training rows (%.0f s)"
            % (n, n, seed, info["iterations"], F.shape[0], time.perf_counter() - t_start))
        del xs, c
        return F, T

    Fs, Ts = [], []
    for seed in range(4100, 4108):
        F, T = collect(12, seed, 2048)
        Fs.append(F)
        Ts.append(T)
    for seed in range(4200, 4204):
        F, T = collect(14, seed, 4096)
        Fs.append(F)
        Ts.append(T)
    Fv, Tv = collect(14, 4204, 4096)
    F = torch.cat(Fs).contiguous()
    T = torch.cat(Ts).contiguous()
    nrows = int(F.shape[0])
    del Fs, Ts
    Fv_h, Tv_h = Fv.cpu().numpy(), Tv.cpu().numpy()
    c16 = context(16, 4)
    c16.mlp_set_params(mlp_init(12))
    val0, _ = c16.mlp_loss_grad(Fv_h, Tv_h)
    t0 = time.perf_counter()
    hist = c16.mlp_train(F, T, epochs=args.mlp_epochs, batch=8192, lr=2e-3, seed=3)
    t_train = time.perf_counter() - t0
    val1, _ = c16.mlp_loss_grad(Fv_h, Tv_h)
    params = c16.mlp_get_params()
    log("[mlp] trained on %d rows, %d epochs in %.1f s: training loss %.4f -> %.4f, validation %.4f -> %.4f"
        % (F.shape[0], args.mlp_epochs, t_train, hist[0], hist[-1], val0, val1))
    del F, T

    # held-out CAS(14,14): FP64 sigma, Olsen against the learned preconditioner
    c14 = context(14, 4204)
    c14.mlp_set_params(params)
    held = {}
    for pc in ("olsen", "mlp"):
        t0 = time.perf_counter()
        E, _, info = c14.davidson(k, 1e-10, precond=pc, vectors=False, max_iter=2000)
        held[pc] = {"iterations": info["iterations"], "sigma_calls": info["sigma_calls"],
                    "seconds": time.perf_counter() - t0, "converged": info["converged"],
                    "mlp_fallbacks": info["mlp_fallbacks"], "energies": E.tolist()}
        log("[mlp] CAS(14,14) seed 4204, %s: %d iterations, %.1f s" % (pc, info["iterations"], held[pc]["seconds"]))
    del c14

    # CAS(16,16), the headline's mixed-precision solver with each preconditioner
    runs = {}
    for pc in ("olsen", "mlp"):
        kw = dict(HEADLINE)
        kw["precond"] = pc
        t0 = time.perf_counter()
        E, _, info = c16.davidson(k, 1e-10, vectors=False, history=4000, max_iter=4000,
                                  progress=progress_printer("cas16-" + pc), **kw)
        runs[pc] = (E, info, time.perf_counter() - t0)
    Eref = runs["olsen"][0]
    out = {}
    for pc, (E, info, dt) in runs.items():
        t_hit, it_hit = time_to_threshold(info["hist_energy"], info["hist_time_ms"], Eref)
        out[pc] = {"iterations": info["iterations"], "sigma_calls": info["sigma_calls"], "seconds": dt,
                   "time_to_1e8_s": t_hit, "threshold_iteration": it_hit, "converged": info["converged"],
                   "mlp_fallbacks": info["mlp_fallbacks"], "energies": E.tolist(),
                   "max_energy_difference_vs_olsen": float(np.abs(E - Eref).max())}
        log("[mlp] CAS(16,16) %s: %d iterations, %.1f s, time-to-1e-8 %.1f s" % (pc, info["iterations"], dt, t_hit))
    gain = out["olsen"]["time_to_1e8_s"] / out["mlp"]["time_to_1e8_s"] if out["mlp"]["time_to_1e8_s"] > 0 else None
    print(json.dumps({"metric": "learned preconditioner vs Olsen, CAS(16,16) time-to-1e-8 Eh",
                      "value": gain, "unit": "x (Olsen time / learned time)", "n_gpus": 1,
                      "higher_is_better": True, "data": "synthetic",
                      "config": {"workload": "train CAS(12,12) seeds 4100-4107 + CAS(14,14) seeds 4200-4203, "
                                             "validate CAS(14,14) seed 4204, apply CAS(16,16) seed 4, 3 roots",
                                 "network": "8-64-64-1 tanh, FP32", "epochs": args.mlp_epochs},
                      "training": {"rows": nrows, "validation_rows": int(Fv_h.shape[0]), "loss_first_epoch": float(hist[0]),
                                   "loss_last_epoch": float(hist[-1]), "validation_loss_before": val0,
                                   "validation_loss_after": val1, "seconds": t_train},
                      "held_out_cas14": held, "cas16": out}), flush=True)


def kernel_figures(P, dims, n, tag, full=False):
    """Per-launch averages and rates of the sigma kernels from HIP events recorded
    on the library's stream (P = profile_read()[tag]). full: the alpha-beta term
    runs over all n^2 ordered pairs (dressed integrals, S^2 penalty)."""
    nb_sig = P["sigma_builds"]
    if nb_sig <= 0:
        return None
    Nd = dims["Ndet"]
    M = n * n if full else n * (n + 1) // 2
    ab_flops = 2.0 * M * dims["sa"] * Nd
    ab_ms = P["ab_ms"] / nb_sig
    cv_ms = P.get("convert_ms", 0.0) / nb_sig
    aa_ms = P["aa_ms"] / nb_sig - cv_ms  # the gather launch alone
    esz = 8 if tag == "f64" else 4
    # one same-spin gather launch: read C, write sigma in FP64, read the
    # operator rows (16-bit columns and values in the input's type)
    gather_bytes = Nd * esz + Nd * 8.0 + dims["Na"] * dims["ra"] * (2.0 + esz)
    gathered = dims["ra"] * Nd * float(esz)
    # one FP64 multiply-add per operator entry and column (the diagonal included)
    gather_flops = 2.0 * dims["ra"] * Nd
    peak = PEAK["%s_TF" % ("f64" if tag == "f64" else HEADLINE["ab_prec"])]
    return {
        "sigma_builds": int(nb_sig),
        "ms_per_sigma": P["total_ms"] / nb_sig,
        "alpha_alpha_gather_ms": aa_ms, "convert_ms": cv_ms, "beta_beta_ms": P["bb_ms"] / nb_sig,
        "combine_ms": P["combine_ms"] / nb_sig,
        "alpha_beta_ms": ab_ms,
        "alpha_beta_TFLOPs": ab_flops / (ab_ms * 1e-3) / 1e12,
        "alpha_beta_mfma_util": ab_flops / (ab_ms * 1e-3) / 1e12 / peak,
        "alpha_beta_flops": ab_flops,
        "gather_GBps_algorithmic": gather_bytes / (aa_ms * 1e-3) / 1e9,
        "gather_GBps_gathered_operands": gathered / (aa_ms * 1e-3) / 1e9,
        "gather_bytes_algorithmic": gather_bytes,
        "gather_flops": gather_flops,
        "gather_TFLOPs": gather_flops / (aa_ms * 1e-3) / 1e12,
    }


def elements_per_sigma(n, na, nb):
    """Matrix elements the oracle evaluates for one matrix-free sigma: every
    determinant with itself, its single and its double substitutions that keep
    the numbers of alpha and beta electrons."""
    sa, sb = na * (n - na), nb * (n - nb)
    daa = math.comb(na, 2) * math.comb(n - na, 2)
    dbb = math.comb(nb, 2) * math.comb(n - nb, 2)
    return math.comb(n, na) * math.comb(n, nb) * (1 + sa + sb + daa + dbb + sa * sb)


def blas_info():
    try:
        from threadpoolctl import threadpool_info
        libs = [x for x in threadpool_info() if x.get("user_api") == "blas"]
        if libs:
            return "%s %s (%s threads)" % (libs[0].get("internal_api"), libs[0].get("version"),
                                          libs[0].get("num_threads"))
    except Exception:
        pass
    return "unknown"


def cpu_leg(seconds, full=False):
    """The CPU oracle timed on this host's cores (tiers of the CPU baseline plan):
    T0 dense Slater-Condon H + LAPACK eigensolver at CAS(6,6) and CAS(8,8); T2
    the matrix-free Slater-Condon sigma at CAS(12,12), rows dealt to one thread
    per core until `seconds` run out (all of sigma if it finishes). full=True
    adds T0 at the CAS(9,9) doublet and T1 (sparse H + Lanczos, eigsh) at
    CAS(10,10), minutes of work."""
    from concurrent.futures import ThreadPoolExecutor
    import threading
    import oracle
    from paper_2405_10197_amd import synth
    cores = len(os.sched_getaffinity(0))
    out = {"cores": cores, "blas": blas_info(), "tiers": {}}
    t0_cases = [(6, 3, 3, 1), (8, 4, 4, 3000)] + ([(9, 5, 4, 3001)] if full else [])
    for n, na, nb, seed in t0_cases:
        h, eri, _ = synth.integrals(n, seed)
        t0 = time.perf_counter()
        H = oracle.hamiltonian(h, eri, na, nb)
        w = np.linalg.eigvalsh(H)
        dt = time.perf_counter() - t0
        out["tiers"]["T0_cas%d" % n] = {"method": "dense H + LAPACK eigvalsh", "determinants": int(H.shape[0]),
                                       "seconds": dt, "E0": float(w[0])}
        del H
        log("[cpu] T0 CAS(%d,%d): %.2f s" % (n, n, dt))
    if full:
        import scipy.sparse.linalg as sla
        h, eri, _ = synth.integrals(10, 3002)
        t0 = time.perf_counter()
        Hs = oracle.hamiltonian_csr(h, eri, 5, 5)
        w = np.sort(sla.eigsh(Hs, k=4, which="SA", tol=1e-13)[0])
        dt = time.perf_counter() - t0
        out["tiers"]["T1_cas10"] = {"method": "sparse H + eigsh", "determinants": int(Hs.shape[0]),
                                    "nonzeros": int(Hs.nnz), "seconds": dt, "E": w.tolist()}
        del Hs
        log("[cpu] T1 CAS(10,10): %.1f s" % dt)
    # T2: matrix-free sigma at CAS(12,12), one thread per core (the C oracle
    # releases the interpreter lock while it runs)
    n, ne = 12, 6
    h, eri, _ = synth.integrals(n, 2)
    Na = math.comb(n, ne)
    Nd = Na * Na
    C = synth.ci_vector(Na, Na, 8)[0]
    order = np.random.default_rng(7).permutation(Nd)
    chunk = 2048
    lock = threading.Lock()
    state = {"next": 0, "rows": 0}
    deadline = time.perf_counter() + seconds

    def worker():
        while time.perf_counter() < deadline:
            with lock:
                i = state["next"]
                state["next"] = i + chunk
            if i >= Nd:
                return
            rows = order[i:i + chunk]
            oracle.sigma_rows(h, eri, ne, ne, C, rows)
            with lock:
                state["rows"] += rows.size

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        for f in [ex.submit(worker) for _ in range(cores)]:
            f.result()
    dt = time.perf_counter() - t0
    rows = state["rows"]
    t_sigma12 = dt * Nd / max(rows, 1)
    out["tiers"]["T2_cas12"] = {"method": "matrix-free Slater-Condon sigma, %d threads" % cores,
                                "determinants": Nd, "rows_done": rows, "seconds": dt,
                                "seconds_per_sigma": t_sigma12, "measured_whole_sigma": rows >= Nd}
    log("[cpu] T2 CAS(12,12): %d of %d rows in %.1f s on %d threads -> %.1f s per sigma"
        % (rows, Nd, dt, cores, t_sigma12))
    out["t_sigma12"] = t_sigma12
    return out


def headline(args):
    """The headline metric: time-to-1e-8 Eh of the mixed-precision solver against
    the FP64 diagonal-preconditioned solve, with roofline and CPU figures."""
    import torch
    from paper_2405_10197_amd import casci, synth

    n, na, nb, k, seed, spin, desc = WORKLOADS[args.workload]
    h, eri, e_core = workload_integrals(args.workload, n, seed)
    common = dict(spin=spin, s2_penalty=1.0 if spin == "singlet" else 0.0)
    cpu = None if args.no_cpu_baseline else cpu_leg(args.cpu_seconds, full=args.cpu_full)

    # baseline and reference: plain FP64 sigma, diagonal preconditioner, residual < 1e-7
    log("[bench] FP64 diagonal-preconditioned solve of %s (reference energies, |r| < 1e-7)" % args.workload)
    bctx = make_ctx(casci, h, eri, n, na, nb, e_core)
    dims = bctx.dims
    bctx.profile(True)
    t0 = time.perf_counter()
    Eref, _, ib = bctx.davidson(k, 1e-10, r_tol=1e-7, vectors=False, history=4000, precond="diag", max_iter=4000,
                                progress=progress_printer("fp64-diag"), **common)
    t_ref = time.perf_counter() - t0
    base_prof = bctx.profile_read()
    t_base, it_base = time_to_threshold(ib["hist_energy"], ib["hist_time_ms"], Eref)
    log("[bench] reference: converged %s, %d iterations, %.1f s, time-to-1e-8 %.2f s, max |r| %.1e" %
        (ib["converged"], ib["iterations"], t_ref, t_base, max(ib["residual"])))
    del bctx
    torch.cuda.empty_cache()

    # headline solver: warm-up and timed steps inside the wall-clock budget
    if args.m_max:
        HEADLINE["m_max"] = args.m_max
    if args.ab_prec:
        HEADLINE["ab_prec"] = args.ab_prec
    budget_end = T_START + args.budget_s
    est = 0.8 * t_ref  # a step is the faster solve; refined by the measured steps
    times, ttt, infos, profs, Es = [], [], [], [], []
    ran_w = ran_t = 0
    # Timed steps come first: one warm-up if the budget leaves room for it and a
    # timed step, more only where every requested timed step still fits.
    n_fit = int((budget_end - time.time()) // est)
    w_plan = min(args.warmup, max(0, n_fit - args.steps), n_fit - 1)
    if args.warmup > 0 and n_fit >= 2:
        w_plan = max(w_plan, 1)
    w_plan = max(w_plan, 0)
    if w_plan < args.warmup:
        log("[bench] budget: %d of %d warm-up steps (about %d steps fit)" % (w_plan, args.warmup, n_fit))
    while True:
        remaining = budget_end - time.time()
        if ran_w < w_plan:
            warm = True
        elif ran_t < args.steps:
            if ran_t >= 1 and remaining < est:
                log("[bench] budget: %d of %d timed steps (%.0f s left, a step takes %.0f s)"
                    % (ran_t, args.steps, remaining, est))
                break
            warm = False
        else:
            break
        tag = "warmup%d" % ran_w if warm else "step%d" % ran_t
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = make_ctx(casci, h, eri, n, na, nb, e_core)
        ctx.profile(True)
        E, _, info = ctx.davidson(k, 1e-10, vectors=False, history=4000, max_iter=4000,
                                  progress=progress_printer(tag), **HEADLINE, **common)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = ctx.profile_read()
        tuning = ctx.tuning()
        del ctx
        est = max(est if (ran_w + ran_t) else 0.0, 1.05 * dt)
        t_hit, it_hit = time_to_threshold(info["hist_energy"], info["hist_time_ms"], Eref)
        log("[bench] %s: %.2f s, time-to-1e-8 %.2f s (iteration %d), %d iterations, %d sigma (%d FP64)" %
            (tag, dt, t_hit, it_hit, info["iterations"], info["sigma_calls"], info["sigma_calls_fp64"]))
        if warm:
            ran_w += 1
        else:
            ran_t += 1
            times.append(dt)
            ttt.append(t_hit)
            infos.append(info)
            profs.append(prof)
            Es.append(E)
    E = Es[-1]
    info = infos[-1]
    P = profs[-1]
    full = args.workload.startswith("dressed") or spin == "singlet"
    lowp = kernel_figures(P["lowp"], dims, n, "lowp", full)
    f64 = kernel_figures(P["f64"], dims, n, "f64", full)
    f64_base = kernel_figures(base_prof["f64"], dims, n, "f64", full)
    # dominant kernel of the timed step (total device time)
    cand = []
    for tag, fig in (("lowp", lowp), ("f64", f64)):
        if fig:
            nbld = fig["sigma_builds"]
            cand.append((fig["alpha_beta_ms"] * nbld, tag, "ab", fig))
            cand.append((fig["alpha_alpha_gather_ms"] * nbld, tag, "aa", fig))
    cand.sort(key=lambda c: -c[0])
    _, tag, part, fig = cand[0]
    device_time_s = {"%s_%s" % (t, p): round(ms / 1000.0, 3) for ms, t, p, _ in cand}
    if part == "ab":
        lp = HEADLINE["ab_prec"]
        peak = PEAK["%s_TF" % lp] if tag == "lowp" else PEAK["f64_TF"]
        # BF16: the fixed-point row kernel (the beta space fits its 16-bit targets here)
        # all ordered pairs (dressed integrals, S^2 penalty): the table-driven kernel
        kname = {"bf16": "k_ab_lp<MfmaBF16>" if full else "k_ab_bf16<double,3,3>",
                 "f32": "k_ab_lp<MfmaF32>"}.get(lp, "k_ab<MfmaF64>") if tag == "lowp" else "k_ab<MfmaF64>"
        ach = fig["alpha_beta_TFLOPs"]
        traffic = read_traffic(os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (
            {"bf16": "ab_bf16", "f32": "ab_lp_f32"}.get(lp, "ab_f64") if tag == "lowp" else "ab_f64",
            args.workload)))
        roof = {"kernel": kname, "bound": "mfma", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": traffic}
    else:
        # the width the autotuner chose for this space (99: row-blocked LDS form)
        code = tuning.get("f32in" if tag == "lowp" else "f64", 0)
        blocked = code == 99
        # the BF16 build's row-blocked gather sums in FP32 (FP32 vector roof),
        # every other build in FP64
        acc32 = tag == "lowp" and blocked and HEADLINE["ab_prec"] == "bf16"
        # (the last template argument: rows per wave, 2 with the 32-row blocks
        # that CAS(16,16)'s unions fit; FP64 sums of column pairs take 1)
        if tag == "lowp":
            kname = ("k_ss_gather_blk<float,double,float,2,%s>" % ("float,2" if acc32 else "double,1")
                     if blocked else "k_ss_gather<float,double>")
            pmc = "ss_gather_blk_f32" if blocked else "ss_gather_f32"
        else:
            kname = "k_ss_gather_blk<double,double,double,1,double,2>" if blocked else "k_ss_gather<double,double>"
            pmc = "ss_gather_blk_f64" if blocked else "ss_gather_f64"
        traffic = read_traffic(os.path.join(ROOT, "profiles", "%s_%s_pmc.txt" % (pmc, args.workload)))
        # Roofline: the compulsory bytes (read C once, write sigma, read the
        # operator) take a fraction of a millisecond at 8 TB/s, the
        # multiply-adds several: the binding roof is the vector rate of the
        # accumulation type
        ach = fig["gather_TFLOPs"]
        vpeak = PEAK["f32_TF"] if acc32 else PEAK["f64_TF"]
        roof = {"kernel": kname, "width_code": code, "bound": "alu", "achieved": ach, "peak": vpeak,
                "unit": "TFLOP/s", "frac": ach / vpeak, "traffic": traffic,
                "hbm_view": {"achieved_GBps": fig["gather_GBps_algorithmic"], "peak_GBps": PEAK["hbm_GBps"],
                             "frac": fig["gather_GBps_algorithmic"] / PEAK["hbm_GBps"]}}
    # the counters' HBM-side bytes over the same launch time (what the memory
    # side actually moved, against the algorithmic bytes of 'achieved')
    t_ms = fig["alpha_beta_ms"] if part == "ab" else fig["alpha_alpha_gather_ms"]
    roof["traffic_GBps"] = traffic / (t_ms * 1e-3) / 1e9 if traffic else None

    med = float(np.median(ttt))
    it_hit = time_to_threshold(info["hist_energy"], info["hist_time_ms"], Eref)[1]
    cpu_baseline = None
    if cpu is not None:
        # the oracle's sigma at this size, from its measured CAS(12,12) rate scaled by
        # the matrix elements per sigma, times the sigma builds the timed solve needed
        # up to the iteration at which it reached 1e-8 Eh
        scale = elements_per_sigma(n, na, nb) / elements_per_sigma(12, 6, 6)
        t_sig = cpu["t_sigma12"] * scale
        nsig = info["sigma_calls"] * (it_hit + 1) / max(info["iterations"], 1) if it_hit >= 0 else info["sigma_calls"]
        cpu_baseline = {
            "value": t_sig * nsig, "unit": "s", "cores": cpu["cores"], "kind": "oracle",
            "sample": "matrix-free Slater-Condon sigma of the oracle at CAS(12,12) on %d threads (%d of %d "
                      "rows in %.1f s), scaled by the matrix elements per sigma to %s (x%.0f) and by the %.0f "
                      "sigma builds the timed solve needed to reach 1e-8 Eh: an extrapolation, not a CPU run "
                      "at this size" % (cpu["cores"], cpu["tiers"]["T2_cas12"]["rows_done"],
                                        cpu["tiers"]["T2_cas12"]["determinants"],
                                        cpu["tiers"]["T2_cas12"]["seconds"], args.workload, scale, nsig),
            "oracle_seconds_per_sigma": t_sig, "blas": cpu["blas"], "tiers": cpu["tiers"],
        }
    s2 = [float(x) for x in info["s2"]]
    spins = [0.5 * (math.sqrt(1.0 + 4.0 * max(x, 0.0)) - 1.0) for x in s2]
    w = np.full(k, 1.0 / k)
    out = {
        "metric": METRIC, "value": med, "unit": "s", "n_gpus": 1, "steps": ran_t, "warmup": ran_w,
        "steps_requested": args.steps_requested, "warmup_requested": args.warmup_requested,
        "budget_s": args.budget_s, "ms_per_step": 1000.0 * float(np.mean(times)), "higher_is_better": False,
        "scaling": "strong", "vs_baseline": None, "dtype": "%s+f64" % HEADLINE["ab_prec"], "data": "synthetic",
        "config": {"workload": desc, "norb": n, "nalpha": na, "nbeta": nb, "nroots": k, "seed": seed,
                   "spin": spin, "solver": "%s alpha-beta (%s) for corrections + FP64 sigma of the Ritz "
                                           "vectors at each collapse, Olsen, m_max %d"
                   % (HEADLINE["ab_prec"].upper(), "FP32 accumulate" if HEADLINE["ab_prec"] != "f64" else "FP64",
                      HEADLINE["m_max"])},
        "roofline": roof,
        "cpu_baseline": cpu_baseline,
        "fp64_diag_time_to_1e8_s": t_base, "fp64_diag_total_s": t_ref,
        "fp64_diag_iterations": ib["iterations"], "fp64_diag_sigma_calls": ib["sigma_calls"],
        "fp64_diag_max_residual": float(max(ib["residual"])),
        "speedup_vs_fp64_diag": (t_base / med) if med > 0 else None,
        "time_to_1e8_s_all_steps": ttt,
        "iterations": info["iterations"], "threshold_iteration": int(it_hit), "sigma_calls": info["sigma_calls"],
        "sigma_calls_fp64": info["sigma_calls_fp64"], "switch_iteration": info["switch_iter"],
        "energies": E.tolist(), "energies_fp64_reference": Eref.tolist(),
        "energy_state_averaged": float(w @ E), "energy_state_averaged_reference": float(w @ Eref),
        "energy_error_vs_fp64_reference": float(np.abs(E - Eref).max()),
        "s2": s2, "spin_S": spins, "s2_integral": all(abs(S - round(S)) < 1e-6 for S in spins),
        "sigma_fp64": f64_base, "sigma_lowp_" + HEADLINE["ab_prec"]: lowp, "sigma_fp64_in_headline": f64,
        "headline_device_time_s": device_time_s, "refinements": info["refinements"],
        "first_iteration_s": float(info["hist_time_ms"][0]) / 1000.0,
        "fp64_diag_first_iteration_s": float(ib["hist_time_ms"][0]) / 1000.0,
        "setup_s": info["time_setup_ms"] / 1000.0,
        "m_max": HEADLINE["m_max"],
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--budget-s", type=float, default=450.0,
                    help="wall-clock budget from the start of the process: no further step starts once it "
                         "would be exceeded (at least one timed step always runs)")
    ap.add_argument("--workload", default="cas16", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-full", action="store_true", help="also the minutes-long CPU tiers (CAS(9,9) dense, "
                                                          "CAS(10,10) eigsh)")
    ap.add_argument("--m-max", type=int, default=None, help="subspace size of the timed solver (default 48)")
    ap.add_argument("--ab-prec", default=None, choices=["f64", "f32", "bf16"],
                    help="alpha-beta arithmetic of the timed solver's corrections (default bf16)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--sigma-only", default=None, choices=["f64", "f32", "bf16"],
                    help="profiling aid: only run --steps sigma builds of the workload in this precision")
    ap.add_argument("--batch", action="store_true", help="run the batched small-active-space workload instead")
    ap.add_argument("--cas18", action="store_true", help="run the CAS(18,18) FP32-storage sigma workload instead")
    ap.add_argument("--cas18-norb", type=int, default=18, help=argparse.SUPPRESS)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--mlp", action="store_true", help="learned preconditioner at scale: train on CAS(12,12)/"
                                                       "CAS(14,14) solves, compare with Olsen at CAS(16,16)")
    ap.add_argument("--mlp-epochs", type=int, default=8)
    ap.add_argument("--copy-probe", type=float, default=None,
                    help="counter calibration: copy GIB gibibytes once with a plain device copy")
    args = ap.parse_args()
    args.steps_requested, args.warmup_requested = args.steps, args.warmup
    if args.copy_probe:
        import torch
        nb = int(args.copy_probe * (1 << 30))
        a = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": nb, "copy_probe_bytes_written": nb}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the string-CASCI path runs and is measured on exactly one GPU (one MI355X); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        print("bench.py: --steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2405_10197_amd import casci, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.batch:
        batch_mode(args)
        return
    if args.mlp:
        mlp_mode(args)
        return
    if args.cas18:
        cas18_mode(args)
        return
    if args.sigma_only:
        n, na, nb, k, seed, spin, desc = WORKLOADS[args.workload]
        h, eri, e_core = workload_integrals(args.workload, n, seed)
        sigma_only(args, casci, h, eri, n, na, nb, e_core)
        return
    headline(args)


if __name__ == "__main__":
    main()
