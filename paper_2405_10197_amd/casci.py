"""Thin ctypes binding over libcasci.so (C ABI in include/casci.h).

Argument marshalling only: every step of the computation runs in the HIP
library. Host arrays are numpy arrays (the library copies them in and out);
device arrays are torch tensors on the context's GPU, passed by pointer and
used in place on the context's stream (by default torch's current stream).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcasci.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "casci.h")

OK, NOCONV = 0, 1
E_ARG, E_STATE, E_NOMEM, E_DEVICE, E_NONFINITE, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
F64, F32, BF16 = 0, 1, 2
PRECOND = {"diag": 0, "olsen": 1, "mlp": 2}
SPIN = {"any": 0, "singlet": 1}
PREC = {"f64": F64, "f32": F32, "bf16": BF16}
MAX_ROOTS = 32
MLP_NPARAM = 4801

_ERRNAMES = {E_ARG: "E_ARG", E_STATE: "E_STATE", E_NOMEM: "E_NOMEM", E_DEVICE: "E_DEVICE",
             E_NONFINITE: "E_NONFINITE", E_UNSUPPORTED: "E_UNSUPPORTED"}


class CasciError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "?"), code, msg))
        self.code = code


class DavidsonOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int), ("m_max", ctypes.c_int), ("precond", ctypes.c_int),
                ("spin", ctypes.c_int), ("ab_prec", ctypes.c_int), ("refine_rnorm", ctypes.c_double),
                ("r_tol", ctypes.c_double), ("s2_penalty", ctypes.c_double),
                ("guess", ctypes.c_void_p), ("nguess", ctypes.c_int), ("guess_mem", ctypes.c_int),
                ("verbose_history", ctypes.c_int), ("progress", ctypes.c_void_p),
                ("progress_user", ctypes.c_void_p), ("graph", ctypes.c_int), ("buffer_roots", ctypes.c_int)]


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                               ctypes.c_double)


def _make_opts(precond="diag", spin="any", ab_prec="f64", max_iter=0, m_max=0, r_tol=0.0, refine_rnorm=0.0,
               s2_penalty=0.0, progress=None, graph=False, buffer_roots=0):
    """Option struct (and the ctypes callback object, which must stay alive during the call)."""
    o = DavidsonOpts()
    cb = None
    if progress is not None:
        def _cb(user, it, k, th, rn, ms):
            progress(it, [th[i] for i in range(k)], [rn[i] for i in range(k)], ms)
        cb = PROGRESS_FN(_cb)
        o.progress = ctypes.cast(cb, ctypes.c_void_p)
    o.max_iter, o.m_max = int(max_iter), int(m_max)
    o.precond, o.spin, o.ab_prec = PRECOND[precond], SPIN[spin], PREC[ab_prec]
    o.refine_rnorm, o.r_tol, o.s2_penalty = float(refine_rnorm), float(r_tol), float(s2_penalty)
    o.graph = 1 if graph else 0
    o.buffer_roots = int(buffer_roots)
    return o, cb


def _info_dict(info, nroots):
    return {
        "iterations": info.iterations, "sigma_calls": info.sigma_calls,
        "sigma_calls_fp64": info.sigma_calls_fp64, "converged": bool(info.converged),
        "switch_iter": info.switch_iter, "mlp_fallbacks": info.mlp_fallbacks,
        "refinements": info.refinements,
        "residual": list(info.residual[:nroots]), "s2": list(info.s2[:nroots]),
        "time_total_ms": info.time_total_ms, "time_sigma_ms": info.time_sigma_ms,
        "time_setup_ms": info.time_setup_ms,
    }


class DavidsonInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("sigma_calls", ctypes.c_int),
                ("sigma_calls_fp64", ctypes.c_int), ("converged", ctypes.c_int),
                ("switch_iter", ctypes.c_int), ("mlp_fallbacks", ctypes.c_int),
                ("refinements", ctypes.c_int),
                ("residual", ctypes.c_double * MAX_ROOTS), ("s2", ctypes.c_double * MAX_ROOTS),
                ("time_total_ms", ctypes.c_double), ("time_sigma_ms", ctypes.c_double),
                ("time_setup_ms", ctypes.c_double), ("hist_energy", ctypes.c_void_p),
                ("hist_residual", ctypes.c_void_p), ("hist_time_ms", ctypes.c_void_p),
                ("hist_len", ctypes.c_int)]


_lib = None


def header_symbols():
    """Names of every function declared in include/casci.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(casci_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load libcasci.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libcasci.so is not built; run `python -m paper_2405_10197_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sig = {
        "casci_create": (I, [ctypes.POINTER(P), I, P]),
        "casci_destroy": (None, [P]),
        "casci_last_error": (ctypes.c_char_p, [P]),
        "casci_set_integrals": (I, [P, I, P, P, D, I]),
        "casci_build_strings": (I, [P, I, I, I]),
        "casci_get_dims": (I, [P, P]),
        "casci_get_strings": (I, [P, I, P]),
        "casci_get_single_list": (I, [P, I, P, P, P, P]),
        "casci_get_same_spin_operator": (I, [P, I, P, P]),
        "casci_get_diagonal": (I, [P, P, I]),
        "casci_sigma": (I, [P, P, P, I, I, I]),
        "casci_sigma_parity": (I, [P, P, P, I, I, I]),
        "casci_sigma_noalloc": (I, [P, P, P, I, I]),
        "casci_spin_square": (I, [P, P, P, I]),
        "casci_rdm": (I, [P, P, I, P, P]),
        "casci_rdm_spin_free": (I, [P, P, I, P, P]),
        "casci_davidson": (I, [P, I, D, P, P, P, I, P]),
        "casci_profile_enable": (I, [P, I]),
        "casci_mlp_set_params": (I, [P, P, I64, I]),
        "casci_mlp_get_params": (I, [P, P]),
        "casci_mlp_forward": (I, [P, P, I64, P, I]),
        "casci_mlp_loss_grad": (I, [P, P, P, I64, P, P, I]),
        "casci_mlp_train": (I, [P, P, P, I64, I, I, ctypes.c_float, ctypes.c_uint64, P, I]),
        "casci_mlp_collect": (I, [P, I, D, P, P, I, ctypes.c_uint64, P, P, I64, P]),
        "casci_mlp_features": (I, [P, P, P, D, P, I, P]),
        "casci_profile_read": (I, [P, P]),
        "casci_abi_layout": (I, [P, I]),
        "casci_sym_eig": (I, [P, I, P, P]),
        "casci_tile_pairs": (I, [I64, I64, I64, P]),
        "casci_batch_davidson": (I, [P, I, I, D, P, P, P, I]),
        "casci_get_tuning": (I, [P, P]),
        "casci_set_tuning": (I, [P, I, I]),
        "casci_get_ab_layout": (I, [P, P]),
        "casci_lowest_diagonal": (I, [P, ctypes.c_int64, P]),
        "casci_release_cache": (I, [I]),
        "casci_ss_block_tables": (I, [I64, I, P, P, I, P, P, P, P, P, P, P]),
        "casci_cached_bytes": (ctypes.c_int64, [I]),
        "casci_set_ab_layout": (I, [P, I, I]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    lay = (ctypes.c_int64 * 6)()
    if L.casci_abi_layout(lay, 6) != 0:
        raise RuntimeError("casci_abi_layout failed")
    mine = [ctypes.sizeof(DavidsonOpts), ctypes.sizeof(DavidsonInfo), DavidsonOpts.progress.offset,
            DavidsonInfo.residual.offset, DavidsonInfo.hist_energy.offset, DavidsonInfo.hist_len.offset]
    if list(lay) != mine:
        raise RuntimeError("libcasci.so struct layout %s differs from the binding's %s" % (list(lay), mine))
    _lib = L
    return L


def _ptr(a):
    """(pointer, mem flag) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        if not a.flags.c_contiguous:
            raise ValueError("array must be C-contiguous")
        return a.ctypes.data, MEM_HOST
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (MEM_DEVICE if a.is_cuda else MEM_HOST)
    raise TypeError("expected a numpy array or a torch tensor")


def _dtype_name(a):
    return str(a.dtype).split(".")[-1]


class Context:
    """One CASCI problem on one GPU (device=-1: validate-only, no GPU needed)."""

    def _vec(self, a, count, name, dtypes=("float64",), device_only=False):
        """Pointer and memory flag of an array argument after checking its element
        count, dtype and placement: a wrong one would make the kernels read or write
        out of bounds, so it is rejected here, before any library call."""
        if not hasattr(a, "shape") or not hasattr(a, "dtype"):
            raise TypeError("%s must be a numpy array or a torch tensor" % name)
        if _dtype_name(a) not in dtypes:
            raise TypeError("%s must be %s, got %s" % (name, " or ".join(dtypes), _dtype_name(a)))
        n = int(np.prod(tuple(a.shape)))
        if n != int(count):
            raise ValueError("%s has %d elements, expected %d" % (name, n, int(count)))
        if isinstance(a, np.ndarray):
            if device_only:
                raise ValueError("%s must be a device tensor" % name)
        elif getattr(a, "is_cuda", False):
            if self.device < 0 or a.device.index != self.device:
                raise ValueError("%s lives on %s, the context on device %d" % (name, a.device, self.device))
        elif device_only:
            raise ValueError("%s must be a device tensor" % name)
        return _ptr(a)

    def __init__(self, device: int = 0, stream=None, own_stream: bool = False):
        """device -1: validate-only context (no GPU work). stream: HIP stream
        handle for the library's work (default: torch's current stream);
        own_stream=True: the library creates a stream of its own (for
        concurrent solves, e.g. batch_davidson)."""
        self._L = lib()
        self.device = device
        if stream is None and device >= 0 and not own_stream:
            import torch
            with torch.cuda.device(device):
                stream = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        rc = self._L.casci_create(ctypes.byref(h), int(device), ctypes.c_void_p(stream or 0))
        if rc != OK:
            raise CasciError(rc, "casci_create(device=%d) failed" % device)
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.casci_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc, allow=(OK,)):
        if rc in allow:
            return rc
        if rc < 0:
            raise CasciError(rc, self.last_error())
        return rc

    def last_error(self) -> str:
        m = self._L.casci_last_error(self._h)
        return m.decode() if m else ""

    def set_tuning(self, f64: int = 0, f32in: int = 0):
        """Force the lanes per gathered entry (16, 32 or 64; 0: autotune)."""
        self._check(self._L.casci_set_tuning(self._h, int(f64), int(f32in)))

    def tuning(self):
        """Autotuned strip width codes of the same-spin gathers, for FP64 and FP32
        input: {'f64': code, 'f32in': code} (16/32/64 lanes per entry, 128,
        1602, 3202, 1604, 3204, 6404 vector forms, 99 row-blocked; 0: not tuned yet)."""
        out = (ctypes.c_int * 2)()
        self._check(self._L.casci_get_tuning(self._h, out))
        return {"f64": out[0], "f32in": out[1]}

    def set_ab_layout(self, pairs: int, code: int):
        """Force the FP64 alpha-beta layout of pair set `pairs` (0: r <= s,
        1: all ordered pairs): 0 = autotune, else 10 MT + split."""
        self._check(self._L.casci_set_ab_layout(self._h, int(pairs), int(code)))

    def ab_layout(self):
        """Autotuned FP64 alpha-beta layouts {'sym': code, 'full': code} (0: not tuned yet)."""
        out = (ctypes.c_int * 2)()
        self._check(self._L.casci_get_ab_layout(self._h, out))
        return {"sym": out[0], "full": out[1]}

    # -- problem definition -------------------------------------------------
    def set_integrals(self, h, eri, e_core: float = 0.0):
        if isinstance(h, np.ndarray):
            h = np.ascontiguousarray(h, dtype=np.float64)
            eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = h.shape[0]
        if tuple(h.shape) != (n, n) or tuple(eri.shape) != (n, n, n, n):
            raise ValueError("h must be [n,n] and eri [n,n,n,n]")
        ph, mem = _ptr(h)
        pe, mem2 = _ptr(eri)
        if mem != mem2:
            raise ValueError("h and eri must live in the same memory")
        self._check(self._L.casci_set_integrals(self._h, n, ph, pe, float(e_core), mem))
        self._keep = (h, eri)

    def build_strings(self, nalpha: int, nbeta: int, norb: int):
        self._check(self._L.casci_build_strings(self._h, int(nalpha), int(nbeta), int(norb)))

    @property
    def dims(self):
        d = np.zeros(8, dtype=np.int64)
        self._check(self._L.casci_get_dims(self._h, d.ctypes.data))
        keys = ["Na", "Nb", "Ndet", "sa", "sb", "ra", "rb", "norb"]
        return {k: int(v) for k, v in zip(keys, d)}

    # -- introspection ------------------------------------------------------
    def strings(self, spin: int):
        N = self.dims["Nb" if spin else "Na"]
        out = np.zeros(N, dtype=np.uint64)
        self._check(self._L.casci_get_strings(self._h, int(spin), out.ctypes.data))
        return out

    def single_list(self, spin: int):
        d = self.dims
        N, s = (d["Nb"], d["sb"]) if spin else (d["Na"], d["sa"])
        J = np.zeros(N * s, dtype=np.int32)
        sg = np.zeros(N * s, dtype=np.int8)
        p = np.zeros(N * s, dtype=np.uint8)
        q = np.zeros(N * s, dtype=np.uint8)
        self._check(self._L.casci_get_single_list(self._h, int(spin), J.ctypes.data, sg.ctypes.data,
                                                  p.ctypes.data, q.ctypes.data))
        return tuple(a.reshape(N, s) for a in (p, q, J, sg))

    def same_spin_operator(self, spin: int):
        d = self.dims
        N, r = (d["Nb"], d["rb"]) if spin else (d["Na"], d["ra"])
        col = np.zeros(N * r, dtype=np.int32)
        val = np.zeros(N * r, dtype=np.float64)
        self._check(self._L.casci_get_same_spin_operator(self._h, int(spin), col.ctypes.data,
                                                         val.ctypes.data))
        return col.reshape(N, r), val.reshape(N, r)

    def diagonal(self, out=None):
        d = self.dims
        if out is None:
            out = np.zeros((d["Na"], d["Nb"]))
        p, mem = self._vec(out, d["Ndet"], "out")
        self._check(self._L.casci_get_diagonal(self._h, p, mem))
        return out

    def lowest_diagonal(self, want: int):
        """Addresses of the `want` lowest diagonal elements, ascending (ties: lower address)."""
        out = np.zeros(int(want), dtype=np.int64)
        self._check(self._L.casci_lowest_diagonal(self._h, int(want), out.ctypes.data))
        return out

    # -- compute ------------------------------------------------------------
    def sigma(self, C, out=None, ab_prec: str = "f64"):
        """sigma = H C. C: [Na, Nb] float64/float32, numpy (host) or torch (device)."""
        if out is None:
            if isinstance(C, np.ndarray):
                out = np.empty_like(C)
            else:
                import torch
                out = torch.empty_like(C)
        nd = self.dims["Ndet"]
        pc, mem = self._vec(C, nd, "C", ("float64", "float32"))
        ps, mem2 = self._vec(out, nd, "out", ("float64", "float32"))
        if mem != mem2 or _dtype_name(out) != _dtype_name(C):
            raise ValueError("C and out must share memory kind and dtype")
        dtype = F64 if _dtype_name(C) == "float64" else F32
        self._check(self._L.casci_sigma(self._h, pc, ps, dtype, PREC[ab_prec], mem))
        return out

    def sigma_parity(self, C, parity: int, out=None, ab_prec: str = "f64"):
        """sigma = H C for a float64 C with C = parity * C^T (nalpha = nbeta): the
        path the Davidson solver takes (one same-spin gather serves both spins)."""
        if out is None:
            if isinstance(C, np.ndarray):
                out = np.empty_like(C)
            else:
                import torch
                out = torch.empty_like(C)
        nd = self.dims["Ndet"]
        pc, mem = self._vec(C, nd, "C")
        ps, mem2 = self._vec(out, nd, "out")
        if mem != mem2:
            raise ValueError("C and out must share memory kind")
        self._check(self._L.casci_sigma_parity(self._h, pc, ps, PREC[ab_prec], int(parity), mem))
        return out

    def sigma_noalloc(self, C, out, ab_prec: str = "f64", parity: int = 0):
        """sigma = H C into `out` without any allocation by the library (device
        float64 tensors; the library's 64 MiB static scratch holds the work
        buffers). casci_sigma must have run once on this context with the same
        ab_prec (it builds the tables)."""
        nd = self.dims["Ndet"]
        pc, _ = self._vec(C, nd, "C", device_only=True)
        ps, _ = self._vec(out, nd, "out", device_only=True)
        self._check(self._L.casci_sigma_noalloc(self._h, pc, ps, PREC[ab_prec], int(parity)))
        return out

    # -- learned preconditioner ------------------------------------------
    def mlp_set_params(self, params):
        p, mem = _ptr(params)
        if str(params.dtype).split(".")[-1] != "float32" or int(np.prod(params.shape)) != MLP_NPARAM:
            raise ValueError("params must be %d float32 values" % MLP_NPARAM)
        self._check(self._L.casci_mlp_set_params(self._h, p, MLP_NPARAM, mem))

    def mlp_get_params(self):
        out = np.zeros(MLP_NPARAM, dtype=np.float32)
        self._check(self._L.casci_mlp_get_params(self._h, out.ctypes.data))
        return out

    def mlp_forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32)
        Y = np.zeros(X.shape[0], dtype=np.float32)
        self._check(self._L.casci_mlp_forward(self._h, X.ctypes.data, X.shape[0], Y.ctypes.data, MEM_HOST))
        return Y

    def mlp_loss_grad(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float32)
        T = np.ascontiguousarray(T, dtype=np.float32)
        g = np.zeros(MLP_NPARAM, dtype=np.float32)
        loss = ctypes.c_double()
        self._check(self._L.casci_mlp_loss_grad(self._h, X.ctypes.data, T.ctypes.data, X.shape[0], g.ctypes.data,
                                                ctypes.byref(loss), MEM_HOST))
        return loss.value, g

    def mlp_train(self, X, T, epochs=10, batch=4096, lr=1e-3, seed=0):
        """X, T: numpy (host) or torch CUDA tensors. Returns per-epoch training loss."""
        N = int(X.shape[0])
        px, mem = self._vec(X, N * 8, "X", ("float32",))
        pt, mem2 = self._vec(T, N, "T", ("float32",))
        if mem != mem2:
            raise ValueError("X and T must share memory kind")
        hist = np.zeros(epochs)
        self._check(self._L.casci_mlp_train(self._h, px, pt, int(X.shape[0]), int(epochs), int(batch),
                                            float(lr), int(seed), hist.ctypes.data, mem))
        return hist

    def mlp_collect(self, nroots, tol, xstar, samples=2048, seed=0, max_rows=1 << 20, **opts):
        """Training rows (features, targets) from a Davidson run; xstar: torch CUDA [nroots, Na, Nb]."""
        import torch
        px, _ = self._vec(xstar, int(nroots) * self.dims["Ndet"], "xstar", device_only=True)
        F = torch.empty((max_rows, 8), dtype=torch.float32, device="cuda:%d" % self.device)
        T = torch.empty(max_rows, dtype=torch.float32, device="cuda:%d" % self.device)
        o = self._opts(**opts)
        n = ctypes.c_int64()
        rc = self._L.casci_mlp_collect(self._h, int(nroots), float(tol), ctypes.byref(o), px,
                                       int(samples), int(seed), F.data_ptr(), T.data_ptr(), int(max_rows),
                                       ctypes.byref(n))
        self._check(rc, allow=(OK, NOCONV))
        return F[:n.value], T[:n.value]

    def mlp_features(self, x, sx, theta, idx):
        """Features of determinants idx for the Ritz pair (theta, x) with sigma sx (torch CUDA FP64)."""
        nd = self.dims["Ndet"]
        px, _ = self._vec(x, nd, "x", device_only=True)
        ps, _ = self._vec(sx, nd, "sx", device_only=True)
        idx = np.ascontiguousarray(idx, dtype=np.int64).reshape(-1)
        if idx.size and (idx.min() < 0 or idx.max() >= nd):
            raise ValueError("determinant index out of range [0, %d)" % nd)
        F = np.zeros((idx.size, 8), dtype=np.float32)
        self._check(self._L.casci_mlp_features(self._h, px, ps, float(theta),
                                               idx.ctypes.data, idx.size, F.ctypes.data))
        return F

    def _opts(self, precond="diag", spin="any", ab_prec="f64", max_iter=0, m_max=0, r_tol=0.0,
              refine_rnorm=0.0, s2_penalty=0.0):
        o = DavidsonOpts()
        o.max_iter, o.m_max = int(max_iter), int(m_max)
        o.precond, o.spin, o.ab_prec = PRECOND[precond], SPIN[spin], PREC[ab_prec]
        o.refine_rnorm, o.r_tol, o.s2_penalty = float(refine_rnorm), float(r_tol), float(s2_penalty)
        return o

    def profile(self, on: bool = True):
        """Start (reset) or stop per-part device timing of sigma builds."""
        self._check(self._L.casci_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """Per-part device time (ms) of the sigma builds since profile(True), split by
        the arithmetic of the alpha-beta term ('f64' and 'lowp'): alpha-alpha gather
        (with the conversions of C), beta-beta work, alpha-beta contraction, final
        combination and whole build, all from events on the library's stream;
        'convert_ms' is the conversions alone (part of 'aa_ms')."""
        out = np.zeros(16)
        self._check(self._L.casci_profile_read(self._h, out.ctypes.data))
        keys = ["aa_ms", "bb_ms", "ab_ms", "combine_ms", "total_ms", "sigma_builds"]
        res = {}
        for tag, off in (("f64", 0), ("lowp", 6)):
            res[tag] = {k: float(out[off + i]) for i, k in enumerate(keys)}
        res["f64"]["convert_ms"] = 0.0
        res["lowp"]["convert_ms"] = float(out[12])
        res.update({k: res["f64"][k] + res["lowp"][k] for k in keys + ["convert_ms"]})
        return res

    def rdm(self, C, two: bool = True, spin_free: bool = False):
        """Density matrices of a float64 CI vector C (host or device). Spin-resolved:
        (g1[2, n, n], g2[3, n, n, n, n] or None), the blocks (alpha, beta) and
        (alpha-alpha, alpha-beta, beta-beta); spin_free: (gamma[n, n], Gamma[n, n, n, n] or None)."""
        pc, mem = self._vec(C, self.dims["Ndet"], "C")
        n = self.dims["norb"]
        if spin_free:
            o1 = np.zeros((n, n))
            o2 = np.zeros((n, n, n, n)) if two else None
            fn = self._L.casci_rdm_spin_free
        else:
            o1 = np.zeros((2, n, n))
            o2 = np.zeros((3, n, n, n, n)) if two else None
            fn = self._L.casci_rdm
        self._check(fn(self._h, pc, mem, o1.ctypes.data, o2.ctypes.data if two else None))
        return o1, o2

    def spin_square(self, C):
        pc, mem = self._vec(C, self.dims["Ndet"], "C")
        s2 = ctypes.c_double()
        self._check(self._L.casci_spin_square(self._h, pc, ctypes.byref(s2), mem))
        return s2.value

    def davidson(self, nroots: int = 1, tol: float = 1e-10, *, precond: str = "diag", spin: str = "any",
                 ab_prec: str = "f64", max_iter: int = 0, m_max: int = 0, r_tol: float = 0.0,
                 refine_rnorm: float = 0.0, s2_penalty: float = 0.0, guess=None, vectors=True,
                 history: int = 0, vectors_out=None, progress=None, graph: bool = False,
                 buffer_roots: int = 0):
        """Lowest roots by Davidson-Liu. Returns (energies, vectors or None, info dict).

        progress: optional callable(iteration, theta list, residual list, wall_ms),
        called by the library once per iteration. graph: replay every sigma build
        from a captured HIP graph.
        """
        o, cb = _make_opts(precond=precond, spin=spin, ab_prec=ab_prec, max_iter=max_iter, m_max=m_max,
                           r_tol=r_tol, refine_rnorm=refine_rnorm, s2_penalty=s2_penalty, progress=progress,
                           graph=graph, buffer_roots=buffer_roots)
        if guess is not None:
            ng = int(guess.shape[0])
            gp, gm = self._vec(guess, ng * self.dims["Ndet"], "guess")
            o.guess, o.nguess, o.guess_mem = gp, ng, gm
        info = DavidsonInfo()
        hist = None
        if history:
            hist = (np.zeros((history, nroots)), np.zeros((history, nroots)), np.zeros(history))
            info.hist_energy, info.hist_residual, info.hist_time_ms = (h.ctypes.data for h in hist)
            info.hist_len = int(history)
        E = np.zeros(nroots)
        vp, vm = 0, MEM_HOST
        vec = None
        if vectors_out is not None:
            vec = vectors_out
            vp, vm = self._vec(vec, int(nroots) * self.dims["Ndet"], "vectors_out")
        elif vectors:
            d = self.dims
            vec = np.zeros((nroots, d["Na"], d["Nb"]))
            vp, vm = _ptr(vec)
        rc = self._L.casci_davidson(self._h, int(nroots), float(tol), ctypes.byref(o), E.ctypes.data,
                                    ctypes.c_void_p(vp or None), vm, ctypes.byref(info))
        self._check(rc, allow=(OK, NOCONV))
        out = _info_dict(info, nroots)
        out["status"] = rc
        if hist is not None:
            n = min(info.iterations, history)
            out["hist_energy"], out["hist_residual"], out["hist_time_ms"] = (
                hist[0][:n], hist[1][:n], hist[2][:n])
        return E, vec, out


def ss_block_tables(col, val, R: int):
    """Row-blocked tables of a same-spin operator in row form (casci_ss_block_tables,
    host only): col int32 [N, r] (diagonal first, then ascending), val float64
    [N, r]. Returns None when the form is not available, else a dict of arrays
    uni, binfo [blocks, 4], goff, rbase, goffs [groups, 4], gvals [groups, 4]."""
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    N, r = col.shape
    if val.shape != col.shape:
        raise ValueError("col and val must have the same shape")
    L = lib()
    sizes = np.zeros(4, dtype=np.int64)
    z = None
    rc = L.casci_ss_block_tables(N, r, col.ctypes.data, val.ctypes.data, int(R), sizes.ctypes.data, z, z, z, z, z, z)
    if rc != OK:
        raise CasciError(rc, "casci_ss_block_tables failed")
    if sizes[3] == 0:
        return None
    out = {"uni": np.zeros(sizes[0], np.uint16), "binfo": np.zeros((sizes[3], 4), np.int32),
           "goff": np.zeros(sizes[2], np.uint16), "rbase": np.zeros(N, np.int32),
           "goffs": np.zeros((sizes[1], 4), np.uint32), "gvals": np.zeros((sizes[1], 4), np.float64)}
    rc = L.casci_ss_block_tables(N, r, col.ctypes.data, val.ctypes.data, int(R), sizes.ctypes.data,
                                 *(out[k].ctypes.data for k in ("uni", "binfo", "goff", "rbase", "goffs", "gvals")))
    if rc != OK:
        raise CasciError(rc, "casci_ss_block_tables failed")
    return out


def release_cache(device: int = -1):
    """Return the library's cached device blocks (casci_release_cache) to the driver."""
    rc = lib().casci_release_cache(int(device))
    if rc != OK:
        raise CasciError(rc, "casci_release_cache failed")


def cached_bytes(device: int = -1) -> int:
    """Bytes of device memory the library's block cache holds (casci_cached_bytes)."""
    return int(lib().casci_cached_bytes(int(device)))


def batch_davidson(contexts, nroots: int = 1, tol: float = 1e-10, *, nthreads: int = 0, **kw):
    """Independent solves of several contexts, run concurrently by the library
    (casci_batch_davidson). kw: the option keywords of Context.davidson (no
    guess / vectors). Returns (energies [count][nroots], list of info dicts)."""
    ctxs = list(contexts)
    if len(set(id(c) for c in ctxs)) != len(ctxs):
        raise ValueError("a context appears twice")
    L = lib()
    o, cb = _make_opts(**kw)
    n = len(ctxs)
    arr = (ctypes.c_void_p * max(n, 1))(*[c._h for c in ctxs])
    E = np.zeros((n, nroots))
    infos = (DavidsonInfo * max(n, 1))()
    rc = L.casci_batch_davidson(arr, n, int(nroots), float(tol), ctypes.byref(o), E.ctypes.data, infos,
                                int(nthreads))
    if rc < 0:
        msgs = [c.last_error() for c in ctxs]
        raise CasciError(rc, "; ".join(m for m in msgs if m) or "batch_davidson failed")
    out = []
    for i in range(n):
        d = _info_dict(infos[i], nroots)
        d["status"] = OK if infos[i].converged else NOCONV
        out.append(d)
    return E, out


def tile_pairs(nb: int, k0: int = 0, count: int | None = None):
    """Tile pairs (bi, bj) of the parity combination pass for workgroups
    k0 .. k0+count-1 (casci_tile_pairs): int64 array [count, 2]."""
    total = nb * (nb + 1) // 2
    count = total - k0 if count is None else count
    out = np.zeros((max(count, 0), 2), dtype=np.int64)
    rc = lib().casci_tile_pairs(int(nb), int(k0), int(count), out.ctypes.data if count > 0 else None)
    if rc < 0:
        raise CasciError(rc, "casci_tile_pairs failed")
    return out


def sym_eig(A):
    """Eigenpairs of a dense symmetric matrix with the solver's host eigensolver
    (casci_sym_eig): (w ascending, Z with unit eigenvectors as columns)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    if A.ndim != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be square")
    n = A.shape[0]
    w = np.zeros(n)
    Z = np.zeros((n, n))
    rc = lib().casci_sym_eig(A.ctypes.data, n, w.ctypes.data, Z.ctypes.data)
    if rc < 0:
        raise CasciError(rc, "casci_sym_eig failed")
    return w, Z
