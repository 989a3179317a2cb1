"""HODLR-accelerated multifrontal solver for MI355X (gfx950).

Thin ctypes binding over the C ABI in include/mfh.h.  Every step of the
analysis, factorisation, preconditioner apply and GMRES runs in the native
library (host C++ for the symbolic analysis, HIP kernels for everything
numeric).  PyTorch is used only to hold device memory and to name streams:
multi right-hand-side vectors are torch tensors of shape (nrhs, n), float64,
contiguous, i.e. column-major n x nrhs as the ABI expects.

There is no fallback: if libmfh.so is missing or no GPU is visible the calls
raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfh.so")
_lib = None

MF_OK, MF_EINVAL, MF_ENOMEM, MF_EBUDGET, MF_ENOTSPD, MF_ENOCONV, MF_ECAPACITY, MF_EHIP, MF_ESTATE = range(9)
MF_APPLY_SCRATCH_BYTES = 64 << 20   # include/mfh.h: the scratch of mf_apply_noalloc
STATUS_NAMES = ["MF_OK", "MF_EINVAL", "MF_ENOMEM", "MF_EBUDGET", "MF_ENOTSPD", "MF_ENOCONV",
                "MF_ECAPACITY", "MF_EHIP", "MF_ESTATE"]
MF_FP64, MF_FP32 = 0, 1
MF_METHOD_HODLR, MF_METHOD_DENSE = 0, 1
(MF_EXP_PERM, MF_EXP_FRONT, MF_EXP_UPD, MF_EXP_UPD_PTR, MF_EXP_RELMAP, MF_EXP_ASM, MF_EXP_BLOCKS,
 MF_EXP_BDLR_I, MF_EXP_BDLR_IPTR, MF_EXP_BDLR_J, MF_EXP_BDLR_JPTR) = range(11)


class MfOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_c", ctypes.c_int32),
                ("bdlr_depth", ctypes.c_int32), ("bdlr_cap", ctypes.c_int32), ("adaptive", ctypes.c_int32),
                ("rank_cap", ctypes.c_int32), ("uv_bf16", ctypes.c_int32), ("apply_graph", ctypes.c_int32),
                ("sampled", ctypes.c_int32), ("apply_split_chunk", ctypes.c_int32),
                ("apply_split_target", ctypes.c_int32), ("eps", ctypes.c_double), ("stream", ctypes.c_void_p)]


class GmresOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("maxit", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class PcgOpts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int32), ("reserved", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class GmresInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("converged", ctypes.c_int32), ("relres", ctypes.c_double)]


class SymbolicInfo(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "nnz", "nfronts", "nlevels", "max_front", "max_npiv")]


class FactorInfo(ctypes.Structure):
    _fields_ = [("persistent_bytes", ctypes.c_int64), ("peak_bytes", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("nblocks", ctypes.c_int64), ("rank_sum", ctypes.c_int64),
                ("rank_max", ctypes.c_int32), ("dense_fronts", ctypes.c_int32), ("hodlr_fronts", ctypes.c_int32),
                ("status_bits", ctypes.c_int32), ("factor_seconds", ctypes.c_double),
                ("resident_bytes", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("leaf", ctypes.c_int32), ("mem_budget", ctypes.c_int64),
                ("tol", ctypes.c_double), ("factor", MfOpts), ("gmres", GmresOpts),
                ("keep_factors", ctypes.c_int32), ("merge", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters_max", ctypes.c_int32), ("relres_max", ctypes.c_double),
                ("t_queue", ctypes.c_double), ("t_analyze", ctypes.c_double), ("t_factor", ctypes.c_double),
                ("t_solve", ctypes.c_double), ("t_total", ctypes.c_double), ("est_bytes", ctypes.c_int64),
                ("peak_bytes", ctypes.c_int64), ("resident_bytes", ctypes.c_int64), ("group_size", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class MfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else status}: {msg}")
        self.status = status


# (name, restype, argtypes) of every entry point declared in include/mfh.h
_P, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
SIGNATURES = [
    ("mf_opts_default", _I32, [ctypes.POINTER(MfOpts)]),
    ("mf_gmres_opts_default", _I32, [ctypes.POINTER(GmresOpts)]),
    ("mf_analyze", _I32, [_I32, _P, _P, _P, _I32, _I32, ctypes.POINTER(_P)]),
    ("mf_symbolic_merge", _I32, [_P, _I32, ctypes.POINTER(_P)]),
    ("mf_symbolic_get_info", _I32, [_P, ctypes.POINTER(SymbolicInfo)]),
    ("mf_symbolic_export", _I32, [_P, _I32, _P, _I64, ctypes.POINTER(_I64)]),
    ("mf_symbolic_bdlr", _I32, [_P, _I32, _I32]),
    ("mf_symbolic_free", None, [_P]),
    ("mf_factor", _I32, [_P, _P, _D, _I32, ctypes.POINTER(MfOpts), ctypes.POINTER(_P)]),
    ("mf_factor_get_info", _I32, [_P, ctypes.POINTER(FactorInfo)]),
    ("mf_factor_ranks", _I32, [_P, _P, _I64, ctypes.POINTER(_I64)]),
    ("mf_factor_free", None, [_P]),
    ("mf_apply", _I32, [_P, _I32, _P, _P, _P]),
    ("mf_apply_noalloc", _I32, [_P, _I32, _P, _P, _P]),
    ("gmres_solve", _I32, [_P, _I32, _P, _P, _D, ctypes.POINTER(GmresOpts), ctypes.POINTER(GmresInfo)]),
    ("mf_direct_solve", _I32, [_P, _I32, _P, _P, _I32, _P, ctypes.POINTER(GmresInfo)]),
    ("mf_pcg_opts_default", _I32, [ctypes.POINTER(PcgOpts)]),
    ("pcg_solve", _I32, [_P, _I32, _P, _P, _D, ctypes.POINTER(PcgOpts), ctypes.POINTER(GmresInfo)]),
    ("mf_spmv", _I32, [_P, _I32, _P, _P, _P]),
    ("mf_estimate_bytes", _I32, [_P, ctypes.POINTER(MfOpts), _I32, _I32, ctypes.POINTER(_I64),
                                 ctypes.POINTER(_I64)]),
    ("mf_server_opts_default", _I32, [ctypes.POINTER(ServerOpts)]),
    ("mf_server_create", _I32, [ctypes.POINTER(ServerOpts), ctypes.POINTER(_P)]),
    ("mf_server_submit", _I32, [_P, _I32, _P, _P, _P, _P, _I32, _I32, _P, ctypes.POINTER(_I64)]),
    ("mf_server_resolve", _I32, [_P, _I64, _I32, _P, ctypes.POINTER(_I64)]),
    ("mf_server_wait", _I32, [_P, _I64, _P, ctypes.POINTER(RequestInfo)]),
    ("mf_server_release", _I32, [_P, _I64]),
    ("mf_server_memory", _I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    ("mf_server_destroy", None, [_P]),
    ("mf_prof_start", _I32, [ctypes.c_char_p]),
    ("mf_prof_stop", _I32, [ctypes.POINTER(KStat), _I32, ctypes.POINTER(_I32)]),
    ("mf_last_error", ctypes.c_char_p, []),
    # include/mfh_testing.h
    ("mfh_test_mfma_layout", _I32, [_I32, _P, _P, _P]),
    ("mfh_test_gemm", _I32, [_I32, _I32, _I32, _I32, _P, _I32, _I32, _P, _I32, _I32, _P, _I32, _D, _D, _I32, _I32]),
    ("mfh_test_gemm_rows", _I32, [_I32, _I32, _I32, _I32, _P, _I32, _I32, _P, _P, _I32, _I32, _P, _P, _I32, _D, _D,
                                  _I32]),
    ("mfh_test_gemm_fold", _I32, [_I32, _I32, _I32, _I32, _P, _I32, _I32, _P, _I32, _P, _I32, _D, _D, _I32, _I32,
                                  _P, _P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_D)]),
    ("mfh_test_potrf", _I32, [_I32, _I32, _P, _I32, _P, _I32, ctypes.POINTER(_I32)]),
    ("mfh_test_skeleton", _I32, [_I32, _P, _I32, _I32, _I32, _I32, _I32, _P, _I32, _P, _I32, _D, _I32, _I32,
                                 _P, _P, ctypes.POINTER(_I32)]),
    ("mfh_test_inverse", _I32, [_I32, _P, _I32, ctypes.POINTER(_I32)]),
    ("mfh_test_phase2_wait", _I32, [_I64]),
    ("mfh_test_record_block_errors", _I32, [_I32]),
    ("mfh_test_block_errors", _I32, [_P, _P, _I64, ctypes.POINTER(_I64)]),
]


def load():
    """Load libmfh.so (built in-tree); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1410_2697_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != MF_OK:
        raise MfError(status, load().mf_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_opts(**kw) -> MfOpts:
    o = MfOpts()
    _check(load().mf_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        if k == "method":
            v = {"hodlr": MF_METHOD_HODLR, "dense": MF_METHOD_DENSE}.get(v, v)
        if k == "precision":
            v = {"fp64": MF_FP64, "fp32": MF_FP32}.get(v, v)
        setattr(o, k, v)
    return o


class Symbolic:
    """mf_analyze: nested dissection, elimination tree, front index maps."""

    def __init__(self, n: int, rowptr, colind, coords, leaf: int):
        lib = load()
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
        self._colind = np.ascontiguousarray(colind, dtype=np.int32)
        c = np.ascontiguousarray(coords, dtype=np.float64)
        dim = 1 if c.ndim == 1 else c.shape[1]
        self.n = int(n)
        self.leaf = int(leaf)
        h = ctypes.c_void_p()
        _check(lib.mf_analyze(self.n, _ptr(self._rowptr), _ptr(self._colind), _ptr(c), dim, self.leaf,
                              ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_csr(cls, A, coords, leaf):
        return cls(A.n, A.rowptr, A.colind, coords, leaf)

    @classmethod
    def merge(cls, parts):
        """mf_symbolic_merge: the analysis of diag(A_1, ..., A_k); factor it
        with the parts' value arrays concatenated."""
        lib = load()
        arr = (ctypes.c_void_p * len(parts))(*[p.h for p in parts])
        h = ctypes.c_void_p()
        _check(lib.mf_symbolic_merge(arr, len(parts), ctypes.byref(h)))
        self = cls.__new__(cls)
        self.n = sum(p.n for p in parts)
        self.leaf = parts[0].leaf
        self.h = h
        return self

    def info(self) -> dict:
        i = SymbolicInfo()
        _check(load().mf_symbolic_get_info(self.h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in SymbolicInfo._fields_}

    def export(self, what: int) -> np.ndarray:
        lib = load()
        n = ctypes.c_int64()
        _check(lib.mf_symbolic_export(self.h, what, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib.mf_symbolic_export(self.h, what, _ptr(out), out.shape[0], ctypes.byref(n)))
        return out[:n.value]

    def bdlr(self, depth: int, cap: int):
        _check(load().mf_symbolic_bdlr(self.h, depth, cap))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mf_symbolic_free(self.h)
            self.h = None


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _devptr(t, n: int, nrhs: int, name: str):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n * nrhs):
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor of shape (nrhs, n)")
    return ctypes.c_void_p(t.data_ptr())


class Factor:
    """mf_factor: numeric factorisation (HODLR or dense fronts) on the GPU."""

    def __init__(self, sym: Symbolic, vals, eps: float = 1e-4, opts: MfOpts | None = None, stream=None, **kw):
        lib = load()
        o = opts if opts is not None else default_opts(**kw)
        o.stream = _stream_ptr(stream).value
        self.sym = sym
        v = np.ascontiguousarray(vals, dtype=np.float64)
        h = ctypes.c_void_p()
        _check(lib.mf_factor(sym.h, _ptr(v), float(eps), 0, ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self.opts = o

    def info(self) -> dict:
        i = FactorInfo()
        _check(load().mf_factor_get_info(self.h, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in FactorInfo._fields_}

    def ranks(self) -> np.ndarray:
        lib = load()
        n = ctypes.c_int64()
        _check(lib.mf_factor_ranks(self.h, None, 0, ctypes.byref(n)))
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib.mf_factor_ranks(self.h, _ptr(out), out.shape[0], ctypes.byref(n)))
        return out[:n.value]

    def apply(self, r, z, stream=None):
        nrhs = r.shape[0] if r.dim() == 2 else 1
        n = self.sym.n
        _check(load().mf_apply(self.h, nrhs, _devptr(r, n, nrhs, "r"), _devptr(z, n, nrhs, "z"),
                               _stream_ptr(stream)))

    def apply_noalloc(self, r, z, stream=None):
        """mf_apply_noalloc: the same apply with its memory in the library's
        static device scratch (no device allocation)."""
        nrhs = r.shape[0] if r.dim() == 2 else 1
        n = self.sym.n
        _check(load().mf_apply_noalloc(self.h, nrhs, _devptr(r, n, nrhs, "r"), _devptr(z, n, nrhs, "z"),
                                       _stream_ptr(stream)))

    def spmv(self, x, y, stream=None):
        nrhs = x.shape[0] if x.dim() == 2 else 1
        n = self.sym.n
        _check(load().mf_spmv(self.h, nrhs, _devptr(x, n, nrhs, "x"), _devptr(y, n, nrhs, "y"),
                              _stream_ptr(stream)))

    def gmres(self, b, x, tol: float = 1e-10, restart: int = 30, maxit: int = 4000, stream=None,
              raise_on_noconv: bool = True):
        lib = load()
        nrhs = b.shape[0] if b.dim() == 2 else 1
        n = self.sym.n
        o = GmresOpts()
        _check(lib.mf_gmres_opts_default(ctypes.byref(o)))
        o.restart, o.maxit = restart, maxit
        o.stream = _stream_ptr(stream).value
        infos = (GmresInfo * nrhs)()
        st = lib.gmres_solve(self.h, nrhs, _devptr(b, n, nrhs, "b"), _devptr(x, n, nrhs, "x"), float(tol),
                             ctypes.byref(o), infos)
        out = [{"iters": i.iters, "converged": bool(i.converged), "relres": i.relres} for i in infos]
        if st == MF_ENOCONV and not raise_on_noconv:
            return out
        _check(st)
        return out

    def direct_solve(self, b, x, refine: int = 1, stream=None):
        """mf_direct_solve: x = M^{-1} b plus `refine` refinement steps."""
        nrhs = b.shape[0] if b.dim() == 2 else 1
        n = self.sym.n
        infos = (GmresInfo * nrhs)()
        _check(load().mf_direct_solve(self.h, nrhs, _devptr(b, n, nrhs, "b"), _devptr(x, n, nrhs, "x"), int(refine),
                                      _stream_ptr(stream), infos))
        return [{"iters": i.iters, "converged": bool(i.converged), "relres": i.relres} for i in infos]

    def pcg(self, b, x, tol: float = 1e-10, maxit: int = 4000, stream=None, raise_on_noconv: bool = True):
        """pcg_solve: preconditioned conjugate gradients with this factor."""
        lib = load()
        nrhs = b.shape[0] if b.dim() == 2 else 1
        n = self.sym.n
        o = PcgOpts()
        _check(lib.mf_pcg_opts_default(ctypes.byref(o)))
        o.maxit = maxit
        o.stream = _stream_ptr(stream).value
        infos = (GmresInfo * nrhs)()
        st = lib.pcg_solve(self.h, nrhs, _devptr(b, n, nrhs, "b"), _devptr(x, n, nrhs, "x"), float(tol),
                           ctypes.byref(o), infos)
        out = [{"iters": i.iters, "converged": bool(i.converged), "relres": i.relres} for i in infos]
        if st == MF_ENOCONV and not raise_on_noconv:
            return out
        _check(st)
        return out

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.mf_factor_free(self.h)
            self.h = None


def prof_start(names=None):
    """Time every launch of the named device kernels (None: all) with HIP
    events on their launch streams, adding up their algorithmic work."""
    arg = None if not names else ";".join(names if not isinstance(names, str) else [names]).encode()
    _check(load().mf_prof_start(arg))


def prof_stop() -> list:
    """Stop timing; one dict per kernel that ran: name, launches, seconds,
    flops, bytes (algorithmic work summed over its launches)."""
    lib = load()
    cap = 64
    arr = (KStat * cap)()
    n = _I32(0)
    _check(lib.mf_prof_stop(arr, cap, ctypes.byref(n)))
    return [{"name": arr[i].name.decode(), "launches": int(arr[i].launches), "seconds": float(arr[i].seconds),
             "flops": float(arr[i].flops), "bytes": float(arr[i].bytes)} for i in range(min(n.value, cap))]


def estimate_bytes(sym: "Symbolic", nrhs: int = 1, restart: int = 30, opts: MfOpts | None = None, **kw) -> dict:
    """Device bytes of a factorisation before running it (host only)."""
    o = opts if opts is not None else default_opts(**kw)
    pe, pk = _I64(0), _I64(0)
    _check(load().mf_estimate_bytes(sym.h, ctypes.byref(o), int(nrhs), int(restart), ctypes.byref(pe),
                                    ctypes.byref(pk)))
    return {"persistent_bytes": pe.value, "peak_bytes": pk.value}


class Server:
    """Continuous-batching request server of the library (see include/mfh.h,
    "Serving").  submit() analyses on the calling thread and returns a
    ticket; wait() blocks for a ticket and returns (x, info) with x of shape
    (n, nrhs).  Calls release the interpreter lock while they block."""

    def __init__(self, slots: int = 4, leaf: int = 128, mem_budget: int = 0, tol: float = 1e-10,
                 keep_factors: bool = False, restart: int = 30, maxit: int = 4000, merge: int = 1, **factor_kw):
        lib = load()
        o = ServerOpts()
        _check(lib.mf_server_opts_default(ctypes.byref(o)))
        o.slots, o.leaf, o.mem_budget, o.tol = int(slots), int(leaf), int(mem_budget), float(tol)
        o.keep_factors = 1 if keep_factors else 0
        o.merge = int(merge)
        o.factor = default_opts(**factor_kw)
        o.gmres.restart, o.gmres.maxit = int(restart), int(maxit)
        h = ctypes.c_void_p()
        _check(lib.mf_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._n = {}

    def submit(self, A, coords, b) -> int:
        b = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(A.n, -1))
        rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(A.colind, dtype=np.int32)
        va = np.ascontiguousarray(A.vals, dtype=np.float64)
        co = np.ascontiguousarray(coords, dtype=np.float64)
        dim = 1 if co.ndim == 1 else co.shape[1]
        t = _I64(0)
        _check(load().mf_server_submit(self.h, int(A.n), _ptr(rp), _ptr(ci), _ptr(va), _ptr(co), dim,
                                       int(b.shape[1]), _ptr(b), ctypes.byref(t)))
        self._n[t.value] = (A.n, b.shape[1])
        return t.value

    def resolve(self, factor_ticket: int, b) -> int:
        n = self._n[factor_ticket][0]
        b = np.asfortranarray(np.asarray(b, dtype=np.float64).reshape(n, -1))
        t = _I64(0)
        _check(load().mf_server_resolve(self.h, int(factor_ticket), int(b.shape[1]), _ptr(b), ctypes.byref(t)))
        self._n[t.value] = (n, b.shape[1])
        return t.value

    def wait(self, ticket: int, raise_on_error: bool = True):
        n, k = self._n[ticket]
        x = np.zeros((n, k), dtype=np.float64, order="F")
        info = RequestInfo()
        st = load().mf_server_wait(self.h, int(ticket), _ptr(x), ctypes.byref(info))
        d = {f: getattr(info, f) for f, _ in RequestInfo._fields_}
        if st != MF_OK and raise_on_error:
            raise MfError(st, load().mf_last_error().decode())
        return x, d

    def release(self, factor_ticket: int):
        _check(load().mf_server_release(self.h, int(factor_ticket)))

    def memory(self) -> dict:
        u, b = _I64(0), _I64(0)
        _check(load().mf_server_memory(self.h, ctypes.byref(u), ctypes.byref(b)))
        return {"in_use": u.value, "budget": b.value}

    def close(self):
        if getattr(self, "h", None):
            load().mf_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
