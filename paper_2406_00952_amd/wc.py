"""ctypes binding of libwcirc (include/wc.h): argument marshalling only.

Every computation runs in the HIP library.  Tensors passed in must be CUDA
(HIP) float64 tensors, contiguous, on the device the plan was created on;
PyTorch is used only to own device memory and to supply the stream.  If the
shared library has not been built this module raises ImportError on import:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("WC_LIBRARY") or os.path.join(_HERE, "lib", "libwcirc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libwcirc.so not built ({LIB_PATH}); run `python -m paper_2406_00952_amd.build`")

_lib = ctypes.CDLL(LIB_PATH)

# ---- status / enums --------------------------------------------------------
WC_OK, WC_E_ARG, WC_E_SINGULAR_S2, WC_E_NOMEM, WC_E_MAXIT, WC_E_BREAKDOWN = 0, 1, 2, 3, 4, 5
WC_E_NONFINITE, WC_E_CANCELLED, WC_E_ADMISSION, WC_E_UNSUPPORTED, WC_E_HIP, WC_E_INTERNAL = 6, 7, 8, 9, 10, 11
METHODS = {"minres_abs_ps": 0, "minres_pms": 1, "gmres_ps": 2}
PRECISIONS = {"fp64": 0, "mixed": 1}
DISCS = {"fd": 0, "fem": 1}
BCS = {"dirichlet": 0, "neumann": 1}


class WcError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_str(code)} (code {code})")


class _Problem(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int), ("M", ctypes.c_int), ("n", ctypes.c_int),
                ("T", ctypes.c_double), ("theta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("zeta", ctypes.c_double), ("s2_remedy", ctypes.c_double),
                ("a_face_host", ctypes.POINTER(ctypes.c_double)), ("disc", ctypes.c_int),
                ("bc", ctypes.c_int), ("kappa", ctypes.c_double)]


class _Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int), ("precision", ctypes.c_int), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int), ("restart", ctypes.c_int), ("flexible", ctypes.c_int),
                ("mg_max_cycles", ctypes.c_int), ("mg_tol", ctypes.c_double),
                ("graphs", ctypes.c_int), ("lowrank", ctypes.c_int)]


class _KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("restarts", ctypes.c_int),
                ("relres", ctypes.c_double), ("relres_est", ctypes.c_double), ("ms", ctypes.c_double),
                ("mg_cycles_max", ctypes.c_int), ("reorth", ctypes.c_int)]


_vp = ctypes.c_void_p
_lib.wc_status_str.restype = ctypes.c_char_p
_lib.wc_status_str.argtypes = [ctypes.c_int]
_lib.wc_version.restype = ctypes.c_char_p
_lib.wc_opts_default.argtypes = [ctypes.POINTER(_Opts)]
_lib.wc_plan_footprint_bytes.restype = ctypes.c_size_t
_lib.wc_plan_footprint_bytes.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Opts)]
_lib.wc_plan_create.argtypes = [ctypes.POINTER(_Problem), ctypes.POINTER(_Opts), _vp, ctypes.POINTER(_vp)]
_lib.wc_plan_destroy.argtypes = [_vp]
_lib.wc_plan_retarget.argtypes = [_vp, ctypes.POINTER(_Problem), ctypes.POINTER(_Opts)]
_lib.wc_plan_autotune.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                  ctypes.POINTER(ctypes.c_int)]
_lib.wc_plan_set_stream.argtypes = [_vp, _vp]
_lib.wc_plan_set_tiles.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
_lib.wc_plan_set_tiles.restype = ctypes.c_int
_lib.wc_rhs.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.wc_matvec.argtypes = [_vp, _vp, _vp]
_lib.wc_pc_apply.argtypes = [_vp, _vp, _vp]
_lib.wc_recover.argtypes = [_vp, _vp, _vp, _vp, _vp]
_lib.wc_krylov.argtypes = [_vp, _vp, _vp, ctypes.POINTER(_Info)]
_lib.wc_solve.argtypes = [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ctypes.POINTER(_Info)]
_lib.wc_profile.argtypes = [_vp, ctypes.c_int]
_lib.wc_profile_read.argtypes = [_vp, ctypes.POINTER(_KStat), ctypes.c_int]
_lib.wc_profile_read.restype = ctypes.c_int
_u64 = ctypes.c_uint64
_lib.wc_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_vp)]
_lib.wc_server_destroy.argtypes = [_vp]
_lib.wc_server_submit.argtypes = [_vp, ctypes.POINTER(_Problem), ctypes.POINTER(_Opts), _vp, _vp, _vp,
                                  _vp, _vp, _vp, ctypes.POINTER(_u64)]
_lib.wc_server_poll.argtypes = [_vp, _u64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_Info)]
_lib.wc_server_wait.argtypes = [_vp, _u64, ctypes.POINTER(_Info), ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
_lib.wc_server_cancel.argtypes = [_vp, _u64]
_lib.wc_server_bytes_in_use.argtypes = [_vp]
_lib.wc_server_bytes_in_use.restype = ctypes.c_size_t
_lib.wc_server_stats.argtypes = [_vp, ctypes.POINTER(_u64), ctypes.POINTER(ctypes.c_int)]
_lib.wc_server_stats.restype = ctypes.c_int
_vpp = ctypes.POINTER(_vp)
_lib.wc_batch_create.argtypes = [_vpp, ctypes.c_int, ctypes.POINTER(_vp)]
_lib.wc_batch_destroy.argtypes = [_vp]
_lib.wc_batch_pc_apply.argtypes = [_vp, _vpp, _vpp]
_lib.wc_batch_solve.argtypes = [_vp, _vpp, _vpp, _vpp, _vpp, _vpp, ctypes.POINTER(_Info)]
_lib.wc_pc_apply_noalloc.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_int, _vp, _vp, _vp]
_lib.wc_pc_apply_noalloc.restype = ctypes.c_int
_lib.wc_pc_apply_noalloc_limit.restype = ctypes.c_size_t
for _f in ("wc_batch_create", "wc_batch_destroy", "wc_batch_pc_apply", "wc_batch_solve"):
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("wc_server_create", "wc_server_destroy", "wc_server_submit", "wc_server_poll",
           "wc_server_wait", "wc_server_cancel"):
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("wc_plan_retarget", "wc_plan_autotune", "wc_profile", "wc_plan_create", "wc_plan_destroy", "wc_plan_set_stream", "wc_rhs", "wc_matvec",
           "wc_pc_apply", "wc_recover", "wc_krylov", "wc_solve"):
    getattr(_lib, _f).restype = ctypes.c_int

EXPORTED = ["wc_status_str", "wc_opts_default", "wc_plan_footprint_bytes", "wc_plan_create",
            "wc_plan_destroy", "wc_plan_retarget", "wc_plan_autotune", "wc_plan_set_tiles",
            "wc_plan_set_stream", "wc_rhs", "wc_matvec", "wc_pc_apply",
            "wc_recover", "wc_krylov", "wc_solve", "wc_version", "wc_profile", "wc_profile_read",
            "wc_server_create", "wc_server_destroy", "wc_server_submit", "wc_server_poll",
            "wc_server_wait", "wc_server_cancel", "wc_server_bytes_in_use", "wc_server_stats",
            "wc_batch_create",
            "wc_batch_destroy", "wc_batch_pc_apply", "wc_batch_solve", "wc_pc_apply_noalloc",
            "wc_pc_apply_noalloc_limit"]


def status_str(code: int) -> str:
    return _lib.wc_status_str(code).decode()


def version() -> str:
    return _lib.wc_version().decode()


@dataclass
class Info:
    status: int
    iters: int
    restarts: int
    relres: float
    relres_est: float
    ms: float
    mg_cycles_max: int
    reorth: int = 0


def _problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, a_face, disc="fd", bc="dirichlet",
             kappa=1.0):
    pr = _Problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, None,
                  DISCS[disc] if isinstance(disc, str) else int(disc),
                  BCS[bc] if isinstance(bc, str) else int(bc), float(kappa))
    keep = None
    if a_face is not None:
        keep = np.ascontiguousarray(a_face, dtype=np.float64)
        pr.a_face_host = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return pr, keep


def _opts(method, precision, tol, maxit, restart, flexible, mg_max_cycles, mg_tol, graphs=True,
          lowrank=False):
    op = _Opts()
    _lib.wc_opts_default(ctypes.byref(op))
    op.method = METHODS[method] if isinstance(method, str) else int(method)
    op.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    op.tol, op.maxit, op.restart, op.flexible = tol, maxit, restart, int(flexible)
    op.mg_max_cycles, op.mg_tol = mg_max_cycles, mg_tol
    op.graphs = int(bool(graphs))
    op.lowrank = int(bool(lowrank))
    return op


def footprint_bytes(dims, M, n, T=1.0, theta=1.0, gamma=1e-4, zeta=np.pi, s2_remedy=1.0,
                    a_face=None, method="gmres_ps", precision="fp64", tol=1e-8, maxit=500,
                    restart=30, flexible=False, mg_max_cycles=30, mg_tol=1e-10,
                    lowrank=False, disc="fd", bc="dirichlet", kappa=1.0) -> int:
    pr, _keep = _problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, a_face, disc, bc, kappa)
    op = _opts(method, precision, tol, maxit, restart, flexible, mg_max_cycles, mg_tol,
               lowrank=lowrank)
    return int(_lib.wc_plan_footprint_bytes(ctypes.byref(pr), ctypes.byref(op)))


def _ptr(t) -> int:
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 device tensor")
    return t.data_ptr()


class Plan:
    """One problem + solver configuration; owns the library's device workspaces."""

    def __init__(self, dims, M, n, T=1.0, theta=1.0, gamma=1e-4, zeta=np.pi, s2_remedy=1.0,
                 a_face=None, method="gmres_ps", precision="fp64", tol=1e-8, maxit=500,
                 restart=30, flexible=False, mg_max_cycles=30, mg_tol=1e-10, stream=None,
                 graphs=True, lowrank=False, disc="fd", bc="dirichlet", kappa=1.0):
        import torch
        pr, keep = _problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, a_face, disc, bc,
                            kappa)
        op = _opts(method, precision, tol, maxit, restart, flexible, mg_max_cycles, mg_tol, graphs,
                   lowrank)
        if stream is None:
            stream = torch.cuda.current_stream()
        self._stream = stream
        h = _vp()
        code = _lib.wc_plan_create(ctypes.byref(pr), ctypes.byref(op), _vp(stream.cuda_stream),
                                   ctypes.byref(h))
        if code != WC_OK:
            raise WcError(code, "wc_plan_create")
        self._h = h
        self.dims, self.M, self.n = dims, M, n
        self.m = M ** dims
        self.nvec = 2 * n * self.m
        self.method, self.precision = method, precision
        self.restart, self.flexible, self.graphs = restart, flexible, graphs
        self.lowrank = lowrank
        self.disc, self.bc = disc, bc
        self.footprint = int(_lib.wc_plan_footprint_bytes(ctypes.byref(pr), ctypes.byref(op)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.wc_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code, where):
        if code not in (WC_OK,):
            raise WcError(code, where)

    def retarget(self, T=1.0, theta=1.0, gamma=1e-4, zeta=np.pi, s2_remedy=1.0, a_face=None,
                 tol=1e-8, maxit=500, mg_max_cycles=30, mg_tol=1e-10, kappa=1.0):
        """Same sizes and method/precision/restart: new problem data, no allocation."""
        pr, _keep = _problem(self.dims, self.M, self.n, T, theta, gamma, zeta, s2_remedy, a_face,
                             self.disc, self.bc, kappa)
        op = _opts(self.method, self.precision, tol, maxit, self.restart, self.flexible,
                   mg_max_cycles, mg_tol, self.graphs, self.lowrank)
        self._check(_lib.wc_plan_retarget(self._h, ctypes.byref(pr), ctypes.byref(op)),
                    "wc_plan_retarget")

    def autotune(self, reps: int = 5):
        """Pick the fastest preconditioner tile widths on this device; returns (ts, tx)."""
        ts, tx = ctypes.c_int(0), ctypes.c_int(0)
        self._check(_lib.wc_plan_autotune(self._h, int(reps), ctypes.byref(ts), ctypes.byref(tx)),
                    "wc_plan_autotune")
        return ts.value, tx.value

    def set_tiles(self, ts: int, tx: int):
        """The preconditioner's kernel choices (values of wc_plan_set_tiles)."""
        self._check(_lib.wc_plan_set_tiles(self._h, int(ts), int(tx)), "wc_plan_set_tiles")

    def set_stream(self, stream):
        self._stream = stream
        self._check(_lib.wc_plan_set_stream(self._h, _vp(stream.cuda_stream)), "wc_plan_set_stream")

    def rhs(self, f, g, y0, b):
        self._check(_lib.wc_rhs(self._h, _ptr(f), _ptr(g), _ptr(y0), _ptr(b)), "wc_rhs")

    def matvec(self, x, y):
        self._check(_lib.wc_matvec(self._h, _ptr(x), _ptr(y)), "wc_matvec")

    def pc_apply(self, v, w):
        self._check(_lib.wc_pc_apply(self._h, _ptr(v), _ptr(w)), "wc_pc_apply")

    def recover(self, x, y, p, u=None):
        self._check(_lib.wc_recover(self._h, _ptr(x), _ptr(y), _ptr(p), _ptr(u)), "wc_recover")

    def krylov(self, b, x, allow_maxit=False) -> Info:
        inf = _Info()
        code = _lib.wc_krylov(self._h, _ptr(b), _ptr(x), ctypes.byref(inf))
        if not (code == WC_OK or (allow_maxit and code == WC_E_MAXIT)):
            raise WcError(code, "wc_krylov")
        return Info(inf.status, inf.iters, inf.restarts, inf.relres, inf.relres_est, inf.ms,
                    inf.mg_cycles_max, inf.reorth)

    def profile(self, enable: bool):
        self._check(_lib.wc_profile(self._h, int(bool(enable))), "wc_profile")

    def profile_read(self) -> dict:
        """{kernel family: (launches, total_ms, algorithmic bytes)} of the last recording."""
        buf = (_KStat * 64)()
        cnt = _lib.wc_profile_read(self._h, buf, 64)
        if cnt < 0:
            raise WcError(WC_E_HIP, "wc_profile_read")
        return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms, buf[i].bytes)
                for i in range(cnt)}

    def solve(self, f, g, y0, y, p, u=None, allow_maxit=False) -> Info:
        inf = _Info()
        code = _lib.wc_solve(self._h, _ptr(f), _ptr(g), _ptr(y0), _ptr(y), _ptr(p), _ptr(u),
                             ctypes.byref(inf))
        if not (code == WC_OK or (allow_maxit and code == WC_E_MAXIT)):
            raise WcError(code, "wc_solve")
        return Info(inf.status, inf.iters, inf.restarts, inf.relres, inf.relres_est, inf.ms,
                    inf.mg_cycles_max, inf.reorth)


def pc_apply_noalloc(v, w, *, dims, M, n, T=1.0, theta=1.0, gamma=1e-4, zeta=np.pi,
                     s2_remedy=1.0, method="gmres_ps", precision="fp64", stream=None,
                     disc="fd", bc="dirichlet", kappa=1.0) -> None:
    """w = P^{-1} v without a plan and without device allocation (wc_pc_apply_noalloc)."""
    import torch
    pr, _keep = _problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, None, disc, bc, kappa)
    if stream is None:
        stream = torch.cuda.current_stream()
    code = _lib.wc_pc_apply_noalloc(ctypes.byref(pr), METHODS[method], PRECISIONS[precision],
                                    _ptr(v), _ptr(w), _vp(stream.cuda_stream))
    if code != WC_OK:
        raise WcError(code, "wc_pc_apply_noalloc")


def pc_apply_noalloc_limit() -> int:
    return int(_lib.wc_pc_apply_noalloc_limit())


def _info(inf) -> Info:
    return Info(inf.status, inf.iters, inf.restarts, inf.relres, inf.relres_est, inf.ms,
                inf.mg_cycles_max, inf.reorth)


def _ptrs(ts):
    return (_vp * len(ts))(*[_ptr(t) for t in ts])


class Batch:
    """Several plans whose preconditioner passes run as one launch per pass (include/wc.h,
    batches).  The plans must stay open, share one stream and not be retargeted while the
    batch exists."""

    def __init__(self, plans):
        self._plans = list(plans)
        arr = (_vp * len(self._plans))(*[p._h for p in self._plans])
        h = _vp()
        code = _lib.wc_batch_create(arr, len(self._plans), ctypes.byref(h))
        if code != WC_OK:
            raise WcError(code, "wc_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib.wc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pc_apply(self, vs, ws):
        code = _lib.wc_batch_pc_apply(self._h, _ptrs(vs), _ptrs(ws))
        if code != WC_OK:
            raise WcError(code, "wc_batch_pc_apply")

    def solve(self, fs, gs, y0s, ys, ps, allow_maxit=False):
        """GMRES(k)-P_S of every instance in lockstep; one Info per instance."""
        infs = (_Info * len(self._plans))()
        code = _lib.wc_batch_solve(self._h, _ptrs(fs), _ptrs(gs), _ptrs(y0s), _ptrs(ys),
                                   _ptrs(ps), infs)
        if not (code == WC_OK or (allow_maxit and code == WC_E_MAXIT)):
            raise WcError(code, "wc_batch_solve")
        return [_info(i) for i in infs]


class Server:
    """Queue of whole solves on worker threads (own HIP streams), admission by the
    plans' device footprint, idle plans cached for reuse (include/wc.h, serving)."""

    def __init__(self, hbm_budget: int = 0, max_concurrency: int = 4):
        h = _vp()
        code = _lib.wc_server_create(ctypes.c_size_t(int(hbm_budget)), int(max_concurrency),
                                     ctypes.byref(h))
        if code != WC_OK:
            raise WcError(code, "wc_server_create")
        self._h = h
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            _lib.wc_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, f, g, y0, y, p, u=None, *, dims, M, n, T=1.0, theta=1.0, gamma=1e-4,
               zeta=np.pi, s2_remedy=1.0, a_face=None, method="gmres_ps", precision="fp64",
               tol=1e-8, maxit=500, restart=30, flexible=False, mg_max_cycles=30,
               mg_tol=1e-10, graphs=True, lowrank=False, disc="fd", bc="dirichlet",
               kappa=1.0) -> int:
        """Queue one solve; the tensors must stay alive and untouched until it is done.
        The server's workers run on their own streams, so the caller's current stream is
        synchronised first: the inputs are complete when the request is queued."""
        import torch
        torch.cuda.current_stream().synchronize()
        pr, keep = _problem(dims, M, n, T, theta, gamma, zeta, s2_remedy, a_face, disc, bc,
                            kappa)
        op = _opts(method, precision, tol, maxit, restart, flexible, mg_max_cycles, mg_tol, graphs,
                   lowrank)
        t = _u64()
        code = _lib.wc_server_submit(self._h, ctypes.byref(pr), ctypes.byref(op), _ptr(f), _ptr(g),
                                     _ptr(y0), _ptr(y), _ptr(p), _ptr(u), ctypes.byref(t))
        if code != WC_OK:
            raise WcError(code, "wc_server_submit")
        self._keep[t.value] = (f, g, y0, y, p, u)
        return t.value

    def poll(self, ticket: int):
        done = ctypes.c_int(0)
        inf = _Info()
        code = _lib.wc_server_poll(self._h, _u64(ticket), ctypes.byref(done), ctypes.byref(inf))
        if code != WC_OK:
            raise WcError(code, "wc_server_poll")
        return (_info(inf) if done.value else None)

    def wait(self, ticket: int):
        """(Info, queue_ms, total_ms); releases the ticket."""
        inf = _Info()
        q, tot = ctypes.c_double(0), ctypes.c_double(0)
        code = _lib.wc_server_wait(self._h, _u64(ticket), ctypes.byref(inf), ctypes.byref(q),
                                   ctypes.byref(tot))
        if code != WC_OK:
            raise WcError(code, "wc_server_wait")
        self._keep.pop(ticket, None)
        return _info(inf), q.value, tot.value

    def cancel(self, ticket: int) -> bool:
        return _lib.wc_server_cancel(self._h, _u64(ticket)) == WC_OK

    def bytes_in_use(self) -> int:
        return int(_lib.wc_server_bytes_in_use(self._h))

    def stats(self):
        """(requests served by continuous batching, largest number active in one round)"""
        b, mx = _u64(0), ctypes.c_int(0)
        self._check_code(_lib.wc_server_stats(self._h, ctypes.byref(b), ctypes.byref(mx)),
                         "wc_server_stats")
        return int(b.value), int(mx.value)

    @staticmethod
    def _check_code(code, where):
        if code != WC_OK:
            raise WcError(code, where)
