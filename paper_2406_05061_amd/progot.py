"""Python binding of libprogot.so (the C ABI declared in include/progot.h).

Argument marshalling only: every step of the path runs in the HIP library.
Tensors must be contiguous float32 CUDA (HIP) tensors on the current device;
work is enqueued on torch's current stream.  PyTorch provides device memory
and the stream handle, nothing else.  There is no CPU fallback: without the
built library every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from dataclasses import dataclass
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
# PROGOT_LIB selects another build of the same library (A/B timing of variants).
LIB_PATH = Path(os.environ.get("PROGOT_LIB", str(_PKG / "libprogot.so")))
HEADER = _PKG.parent / "include" / "progot.h"

POT_OK = 0
POT_WARN_NOT_CONVERGED = 1
POT_BUSY = 2
POT_ERR_INVALID = -1
POT_ERR_NOMEM = -2
POT_ERR_NUMERIC = -3
POT_ERR_DEVICE = -4
PREC = {"fp32": 0, "bf16": 1, "bf16x3": 2}
ALPHA_SCHED = {"constant": 0, "decelerated": 1, "accelerated": 2}
MAX_K = 64


class PotError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


class pot_clouds(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("m", C.c_int64), ("d", C.c_int32), ("precision", C.c_int32),
        ("X", C.c_void_p), ("Y", C.c_void_p), ("a", C.c_void_p), ("b", C.c_void_p),
        ("xk", C.c_void_p),
        ("x_sqn", C.c_void_p), ("y_sqn", C.c_void_p),
        ("log_a", C.c_void_p), ("log_b", C.c_void_p),
        ("x_lp", C.c_void_p), ("y_lp", C.c_void_p), ("yt_lp", C.c_void_p),
        ("mean_cost", C.c_double), ("ws", C.c_void_p), ("ws_bytes", C.c_size_t),
        ("cost_p", C.c_float), ("cmat", C.c_void_p), ("ldc", C.c_int64),
    ]


class pot_sinkhorn_info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("err", C.c_float),
                ("seconds", C.c_double)]


class pot_progot_params(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("alpha_sched", C.c_int32), ("eps_mode", C.c_int32),
        ("theta", C.c_float), ("eps_explicit", C.POINTER(C.c_double)),
        ("tau_first", C.c_float), ("tau_last", C.c_float), ("max_iter", C.c_int32),
        ("warm_start", C.c_int32),
    ]


class pot_progot_info(C.Structure):
    _fields_ = [
        ("K", C.c_int32), ("iters", C.c_int32 * MAX_K), ("converged", C.c_int32),
        ("eps", C.c_float * MAX_K), ("alpha", C.c_float * MAX_K), ("err", C.c_float * MAX_K),
        ("seconds", C.c_double),
    ]


_lib = None
_vp, _i64, _i32, _f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
_SIGS = {
    "pot_workspace_bytes": (C.c_size_t, [_i64, _i64, _i32, _i32]),
    "pot_prepare_clouds": (C.c_int, [C.POINTER(pot_clouds), _vp, _i64, _vp, _i64, _i32, _vp, _vp,
                                     _i32, _vp, C.c_size_t, _vp]),
    "pot_workspace_bytes_pcost": (C.c_size_t, [_i64, _i64, _i32, _f32, _i32]),
    "pot_prepare_clouds_pcost": (C.c_int, [C.POINTER(pot_clouds), _vp, _i64, _vp, _i64, _i32, _vp,
                                           _vp, _f32, _i32, _vp, C.c_size_t, _vp]),
    "pot_sinkhorn_solve": (C.c_int, [C.POINTER(pot_clouds), _f32, _f32, _i32, _vp, _vp, _vp, _vp,
                                     C.POINTER(pot_sinkhorn_info), _vp]),
    "pot_entropic_map": (C.c_int, [C.POINTER(pot_clouds), _vp, _f32, _vp, _i64, _f32, _vp, _vp]),
    "pot_progot_solve": (C.c_int, [C.POINTER(pot_clouds), C.POINTER(pot_progot_params), _vp, _vp,
                                   _vp, C.POINTER(pot_progot_info), _vp]),
    "pot_progot_map": (C.c_int, [C.POINTER(pot_clouds), _i32, _vp, C.POINTER(C.c_float),
                                 C.POINTER(C.c_float), _vp, _i64, _vp, _vp]),
    "pot_marginal_check": (C.c_int, [C.POINTER(pot_clouds), _vp, _vp, _f32, C.POINTER(C.c_double),
                                     _vp]),
    "pot_coupling_metrics": (C.c_int, [C.POINTER(pot_clouds), _vp, _vp, _f32, C.POINTER(C.c_double),
                                       _vp]),
    "pot_diag_metrics": (C.c_int, [C.POINTER(pot_clouds), _vp, _vp, _f32, C.POINTER(C.c_double), _vp]),
    "pot_sinkhorn_divergence_bytes": (C.c_size_t, [_i64, _i64, _i32]),
    "pot_sinkhorn_divergence_pcost_bytes": (C.c_size_t, [_i64, _i64, _i32, _f32]),
    "pot_sinkhorn_divergence_pcost": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _vp, _vp, _f32, _f32, _f32,
                                                _i32, C.POINTER(C.c_double), _vp, C.c_size_t, _vp]),
    "pot_sinkhorn_divergence": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _vp, _vp, _f32, _f32, _i32,
                                          C.POINTER(C.c_double), _vp, C.c_size_t, _vp]),
    "pot_sinkhorn_divergence_noalloc": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _vp, _vp, _f32, _f32,
                                                  _i32, C.POINTER(C.c_double), _vp]),
    "pot_eps_schedule_bytes": (C.c_size_t, [_i64, _i64, _i32, _i32]),
    "pot_eps_schedule_pcost_bytes": (C.c_size_t, [_i64, _i64, _i32, _i32, _f32]),
    "pot_eps_schedule": (C.c_int, [C.POINTER(pot_clouds), _vp, _i64, _i32, _i32,
                                   C.POINTER(C.c_double), _i32, _f32, _f32, _i32,
                                   C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_int32), _vp, C.c_size_t, _vp]),
    "pot_server_arena_overhead": (C.c_size_t, [_i32]),
    "pot_server_request_bytes": (C.c_size_t, [_i64, _i64, _i32]),
    "pot_server_create": (C.c_int, [C.POINTER(C.c_void_p), _vp, C.c_size_t, _i32, _vp]),
    "pot_server_submit": (C.c_int, [_vp, _vp, _i64, _vp, _i64, _i32, C.POINTER(pot_progot_params),
                                    _vp, _vp, _vp, C.POINTER(C.c_int64)]),
    "pot_server_step": (C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "pot_server_poll": (C.c_int, [_vp, C.c_int64, C.POINTER(pot_progot_info)]),
    "pot_server_destroy": (C.c_int, [_vp]),
    "pot_timing_enable": (C.c_int, [C.c_int]),
    "pot_timing_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "pot_status_string": (C.c_char_p, [C.c_int]),
    "pot_version": (C.c_char_p, []),
}


def lib() -> C.CDLL:
    """Load libprogot.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2406_05061_amd.build`")
        L = C.CDLL(str(LIB_PATH))
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_symbols() -> list[str]:
    """Function names declared in include/progot.h."""
    txt = HEADER.read_text()
    return sorted(set(re.findall(r"^POT_API\s+[\w\s\*]*?\b(pot_\w+)\s*\(", txt, flags=re.M)))


def status_string(code: int) -> str:
    return lib().pot_status_string(int(code)).decode()


def version() -> str:
    return lib().pot_version().decode()


PCOST_MODE = {"auto": 0, "on_the_fly": 1, "keep": 2}


def workspace_bytes(n: int, m: int, d: int, precision: str = "fp32", cost_p: float = 0.0,
                    cost_mode: str = "auto") -> int:
    if cost_p:
        if precision != "fp32":
            return 0
        return int(lib().pot_workspace_bytes_pcost(n, m, d, float(cost_p), PCOST_MODE[cost_mode]))
    return int(lib().pot_workspace_bytes(n, m, d, PREC[precision]))


def _check(code: int, where: str, allow_warn: bool = True) -> int:
    if code < 0 or (code > 0 and not allow_warn):
        raise PotError(code, where)
    return code


def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _dev_f32(t, name: str, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Clouds:
    """A prepared pair of clouds: inputs, workspace and the pot_clouds POD.
    Keeps references to every tensor the library points into.  cost_p = 0
    selects the squared-Euclidean cost; cost_p > 1 the cost
    h(z) = (1/p) sum_k |z_k|^p (FP32 only), whose matrix is kept in the
    workspace or formed on the fly per cost_mode ("auto", "keep",
    "on_the_fly")."""

    def __init__(self, X, Y, a=None, b=None, precision: str = "fp32", cost_p: float = 0.0,
                 cost_mode: str = "auto"):
        torch = _torch()
        _dev_f32(X, "X")
        _dev_f32(Y, "Y")
        if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("X (n x d) and Y (m x d) must share d")
        n, d = X.shape
        m = Y.shape[0]
        if a is not None:
            _dev_f32(a, "a", (n,))
        if b is not None:
            _dev_f32(b, "b", (m,))
        nbytes = workspace_bytes(n, m, d, precision, cost_p, cost_mode)
        if nbytes == 0:
            raise PotError(POT_ERR_INVALID, "workspace_bytes")
        self.X, self.Y, self.a, self.b = X, Y, a, b
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        self.c = pot_clouds()
        self.n, self.m, self.d, self.precision = n, m, d, precision
        self.cost_p = float(cost_p)
        if cost_p:
            _check(lib().pot_prepare_clouds_pcost(C.byref(self.c), _ptr(X), n, _ptr(Y), m, d,
                                                  _ptr(a), _ptr(b), float(cost_p),
                                                  PCOST_MODE[cost_mode], _ptr(self.ws), nbytes,
                                                  C.c_void_p(_stream())),
                   "prepare_clouds_pcost", False)
        else:
            _check(lib().pot_prepare_clouds(C.byref(self.c), _ptr(X), n, _ptr(Y), m, d, _ptr(a),
                                            _ptr(b), PREC[precision], _ptr(self.ws), nbytes,
                                            C.c_void_p(_stream())), "prepare_clouds", False)

    @property
    def mean_cost(self) -> float:
        return float(self.c.mean_cost)

    def cost_matrix(self):
        """General costs: a copy of the resident cost matrix C_ij = h(x_i - y_j)
        of the current source iterate (n x m)."""
        if not self.cost_p or not self.c.cmat:
            raise ValueError("these clouds do not keep their cost matrix")
        torch = _torch()
        off = self.c.cmat - self.ws.data_ptr()
        ldc = int(self.c.ldc)
        flat = self.ws[off:off + self.n * ldc * 4].view(torch.float32)
        return flat.view(self.n, ldc)[:, :self.m].clone()

    def xk(self):
        """A copy of the current source iterate X^(k) (n x d), taken on the
        current stream after the library's work."""
        torch = _torch()
        off = self.c.xk - self.ws.data_ptr()
        nbytes = self.n * self.d * 4
        return self.ws[off:off + nbytes].view(torch.float32).view(self.n, self.d).clone()


def prepare_clouds(X, Y, a=None, b=None, precision: str = "fp32", cost_p: float = 0.0,
                   cost_mode: str = "auto") -> Clouds:
    return Clouds(X, Y, a, b, precision, cost_p, cost_mode)


@dataclass
class SinkhornInfo:
    iters: int
    converged: bool
    err: float
    seconds: float
    status: int


def sinkhorn_solve(cl: Clouds, eps: float, tau: float, max_iter: int = 10_000,
                   f_init=None, g_init=None, f=None, g=None):
    """Alg. 1 on the current source iterate; returns (f, g, SinkhornInfo)."""
    torch = _torch()
    dev = cl.X.device
    f = torch.empty(cl.n, dtype=torch.float32, device=dev) if f is None else _dev_f32(f, "f", (cl.n,))
    g = torch.empty(cl.m, dtype=torch.float32, device=dev) if g is None else _dev_f32(g, "g", (cl.m,))
    if f_init is not None:
        _dev_f32(f_init, "f_init", (cl.n,))
    if g_init is not None:
        _dev_f32(g_init, "g_init", (cl.m,))
    info = pot_sinkhorn_info()
    st = _check(lib().pot_sinkhorn_solve(C.byref(cl.c), float(eps), float(tau), int(max_iter),
                                         _ptr(f_init), _ptr(g_init), _ptr(f), _ptr(g),
                                         C.byref(info), C.c_void_p(_stream())), "sinkhorn_solve")
    return f, g, SinkhornInfo(info.iters, bool(info.converged), float(info.err), info.seconds, st)


def entropic_map(cl: Clouds, g, eps: float, Xq, alpha: float = 1.0, out=None):
    """(1 - alpha) Xq + alpha T(Xq) with T the entropic map to cl.Y (eq. Tent)."""
    torch = _torch()
    _dev_f32(g, "g", (cl.m,))
    _dev_f32(Xq, "Xq")
    if Xq.dim() != 2 or Xq.shape[1] != cl.d:
        raise ValueError("Xq must be nq x d")
    out = torch.empty_like(Xq) if out is None else _dev_f32(out, "out", tuple(Xq.shape))
    _check(lib().pot_entropic_map(C.byref(cl.c), _ptr(g), float(eps), _ptr(Xq), Xq.shape[0],
                                  float(alpha), _ptr(out), C.c_void_p(_stream())), "entropic_map",
           False)
    return out


@dataclass
class ProgOTInfo:
    K: int
    iters: list
    converged: bool
    eps: list
    alpha: list
    err: list
    seconds: float
    status: int


def _params(K, alpha_sched="constant", theta=1.0, eps=None, tau_first=1e-3, tau_last=1e-3,
            max_iter=10_000, warm_start="alpha_k"):
    """pot_progot_params plus the buffer its eps pointer refers to (keep both alive)."""
    p = pot_progot_params()
    p.K = int(K)
    p.alpha_sched = ALPHA_SCHED[alpha_sched]
    keep = None
    if eps is None:
        p.eps_mode, p.theta = 0, float(theta)
    else:
        keep = (C.c_double * int(K))(*[float(e) for e in eps])
        p.eps_mode, p.theta, p.eps_explicit = 1, float(theta), C.cast(keep, C.POINTER(C.c_double))
    p.tau_first, p.tau_last = float(tau_first), float(tau_last)
    p.max_iter = int(max_iter)
    p.warm_start = 0 if warm_start == "alpha_k" else 1
    return p, keep


def _info(info, st):
    k = info.K
    return ProgOTInfo(k, list(info.iters[:k]), bool(info.converged), list(info.eps[:k]),
                      list(info.alpha[:k]), list(info.err[:k]), info.seconds, st)


def progot_solve(cl: Clouds, K: int, *, alpha_sched: str = "constant", theta: float = 1.0,
                 eps=None, tau_first: float = 1e-3, tau_last: float = 1e-3,
                 max_iter: int = 10_000, warm_start: str = "alpha_k", want_TX: bool = True):
    """Alg. 2; returns (f, G, TX or None, ProgOTInfo).  eps=None uses the
    per-step mean-cost rule with theta; an array gives an explicit schedule."""
    torch = _torch()
    dev = cl.X.device
    p, keep = _params(K, alpha_sched, theta, eps, tau_first, tau_last, max_iter, warm_start)
    f = torch.empty(cl.n, dtype=torch.float32, device=dev)
    G = torch.empty((K, cl.m), dtype=torch.float32, device=dev)
    TX = torch.empty((cl.n, cl.d), dtype=torch.float32, device=dev) if want_TX else None
    info = pot_progot_info()
    st = _check(lib().pot_progot_solve(C.byref(cl.c), C.byref(p), _ptr(f), _ptr(G), _ptr(TX),
                                       C.byref(info), C.c_void_p(_stream())), "progot_solve")
    del keep
    return f, G, TX, _info(info, st)


def progot_map(cl: Clouds, G, eps, alpha, Xq, out=None):
    """Alg. 3 T_Prog at the rows of Xq (last alpha reset to 1)."""
    torch = _torch()
    K = len(eps)
    _dev_f32(G, "G", (K, cl.m))
    _dev_f32(Xq, "Xq")
    out = torch.empty_like(Xq) if out is None else _dev_f32(out, "out", tuple(Xq.shape))
    e = (C.c_float * K)(*[float(x) for x in eps])
    a = (C.c_float * K)(*[float(x) for x in alpha])
    _check(lib().pot_progot_map(C.byref(cl.c), K, _ptr(G), e, a, _ptr(Xq), Xq.shape[0], _ptr(out),
                                C.c_void_p(_stream())), "progot_map", False)
    return out


@dataclass
class EpsSchedule:
    eps: list          # eps_k for k = 0..K-1 (feed to progot_solve(eps=...))
    errors: list       # hold-out score of each grid scale
    p_star: int        # first argmin of the scores
    status: int


DEFAULT_S_GRID = tuple(2.0 ** p for p in range(-3, 4))


def eps_schedule(cl: Clouds, Y_test, K: int, *, alpha_sched: str = "constant", s_grid=None,
                 beta0: float = 5.0, tau: float = 1e-3, max_iter: int = 10_000) -> EpsSchedule:
    """Alg. 4 (eps-scheduler) on the GPU for the prepared pair ``cl``: grid of
    Y -> Y Sinkhorn solves, hold-out map error, schedule from eps_0 (the
    pair's mean cost / 20) to the selected eps_final."""
    torch = _torch()
    _dev_f32(Y_test, "Y_test")
    if Y_test.dim() != 2 or Y_test.shape[1] != cl.d:
        raise ValueError("Y_test must be m_test x d")
    grid = list(DEFAULT_S_GRID if s_grid is None else s_grid)
    G = len(grid)
    if cl.cost_p:
        nb = int(lib().pot_eps_schedule_pcost_bytes(cl.m, Y_test.shape[0], cl.d, G, cl.cost_p))
    else:
        nb = int(lib().pot_eps_schedule_bytes(cl.m, Y_test.shape[0], cl.d, G))
    if nb == 0:
        raise ValueError("invalid sizes for the eps-scheduler")
    ws = torch.empty(nb, dtype=torch.uint8, device=cl.X.device)
    grid_c = (C.c_double * G)(*[float(v) for v in grid])
    eps_c = (C.c_double * int(K))()
    err_c = (C.c_double * G)()
    p_c = C.c_int32(-1)
    st = _check(lib().pot_eps_schedule(C.byref(cl.c), _ptr(Y_test), Y_test.shape[0], int(K),
                                       ALPHA_SCHED[alpha_sched], grid_c, G, float(beta0), float(tau),
                                       int(max_iter), eps_c, err_c, C.byref(p_c), _ptr(ws), nb,
                                       C.c_void_p(_stream())), "eps_schedule")
    return EpsSchedule(list(eps_c), list(err_c), int(p_c.value), st)


def coupling_metrics(cl: Clouds, f, g, eps: float) -> dict:
    """FP64 metrics of P = exp((f (+) g - C)/eps) on the current source
    iterate: marginal L1 errors, the objective of eq. entdual, <P, C>,
    sum P log P and the mass."""
    _dev_f32(f, "f", (cl.n,))
    _dev_f32(g, "g", (cl.m,))
    out = (C.c_double * 6)()
    _check(lib().pot_coupling_metrics(C.byref(cl.c), _ptr(f), _ptr(g), float(eps), out,
                                      C.c_void_p(_stream())), "coupling_metrics", False)
    return {"row_err": out[0], "col_err": out[1], "ot": out[2], "transport_cost": out[3],
            "p_log_p": out[4], "mass": out[5]}


def diag_metrics(cl: Clouds, f, g, eps: float):
    """(Tr P, KL(I/n || P)) for n == m (coupling-recovery benchmark)."""
    _dev_f32(f, "f", (cl.n,))
    _dev_f32(g, "g", (cl.m,))
    out = (C.c_double * 2)()
    _check(lib().pot_diag_metrics(C.byref(cl.c), _ptr(f), _ptr(g), float(eps), out,
                                  C.c_void_p(_stream())), "diag_metrics", False)
    return out[0], out[1]


def sinkhorn_divergence(X, Y, a=None, b=None, eps: float = 0.0, tau: float = 1e-3,
                        max_iter: int = 10_000, cost_p: float = 0.0) -> dict:
    """Sinkhorn divergence (eq. sink_div); eps = 0 uses 5 % of the mean cost
    within Y (the paper's eps_D); cost_p > 1 evaluates it with the cost
    (1/p)|.|_p^p."""
    torch = _torch()
    for t, nm in ((X, "X"), (Y, "Y")):
        _dev_f32(t, nm)
    n, d = X.shape
    m = Y.shape[0]
    if Y.shape[1] != d:
        raise ValueError("X and Y must have the same dimension")
    if a is not None:
        _dev_f32(a, "a", (n,))
    if b is not None:
        _dev_f32(b, "b", (m,))
    if cost_p:
        nb = int(lib().pot_sinkhorn_divergence_pcost_bytes(n, m, d, float(cost_p)))
    else:
        nb = int(lib().pot_sinkhorn_divergence_bytes(n, m, d))
    if nb == 0:
        raise ValueError("invalid sizes or cost")
    ws = torch.empty(nb, dtype=torch.uint8, device=X.device)
    out = (C.c_double * 5)()
    if cost_p:
        st = _check(lib().pot_sinkhorn_divergence_pcost(
            _ptr(X), n, _ptr(Y), m, d, _ptr(a), _ptr(b), float(cost_p), float(eps), float(tau),
            int(max_iter), out, _ptr(ws), nb, C.c_void_p(_stream())), "sinkhorn_divergence_pcost")
    else:
        st = _check(lib().pot_sinkhorn_divergence(_ptr(X), n, _ptr(Y), m, d, _ptr(a), _ptr(b),
                                                  float(eps), float(tau), int(max_iter), out,
                                                  _ptr(ws), nb, C.c_void_p(_stream())),
                    "sinkhorn_divergence")
    return {"D": out[0], "ot_xy": out[1], "ot_xx": out[2], "ot_yy": out[3], "eps": out[4],
            "status": st}


STATIC_SCRATCH_BYTES = 32 << 20


def sinkhorn_divergence_noalloc(X, Y, a=None, b=None, eps: float = 0.0, tau: float = 1e-3,
                                max_iter: int = 10_000) -> dict:
    """The squared-Euclidean Sinkhorn divergence of ``sinkhorn_divergence``
    computed in the library's static per-GPU scratch array: no workspace
    tensor is allocated, here or in the library."""
    for t, nm in ((X, "X"), (Y, "Y")):
        _dev_f32(t, nm)
    n, d = X.shape
    m = Y.shape[0]
    if Y.shape[1] != d:
        raise ValueError("X and Y must have the same dimension")
    if a is not None:
        _dev_f32(a, "a", (n,))
    if b is not None:
        _dev_f32(b, "b", (m,))
    out = (C.c_double * 5)()
    st = _check(lib().pot_sinkhorn_divergence_noalloc(_ptr(X), n, _ptr(Y), m, d, _ptr(a), _ptr(b),
                                                      float(eps), float(tau), int(max_iter), out,
                                                      C.c_void_p(_stream())),
                "sinkhorn_divergence_noalloc")
    return {"D": out[0], "ot_xy": out[1], "ot_xx": out[2], "ot_yy": out[3], "eps": out[4],
            "status": st}


def marginal_check(cl: Clouds, f, g, eps: float):
    """FP64 (row L1, column L1, dual objective) of the coupling of (f, g) on
    the current source iterate."""
    _dev_f32(f, "f", (cl.n,))
    _dev_f32(g, "g", (cl.m,))
    out = (C.c_double * 3)()
    _check(lib().pot_marginal_check(C.byref(cl.c), _ptr(f), _ptr(g), float(eps), out,
                                    C.c_void_p(_stream())), "marginal_check", False)
    return float(out[0]), float(out[1]), float(out[2])


class Server:
    """Serving form (continuous batching of ProgOT solves; see include/progot.h).

    The arena (a uint8 device tensor) is the HBM budget requests are admitted
    against.  Every call must run with the same current stream as creation."""

    def __init__(self, arena_bytes: int, max_active: int = 64, device="cuda"):
        torch = _torch()
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        self.stream = _stream()
        h = C.c_void_p()
        _check(lib().pot_server_create(C.byref(h), _ptr(self.arena), int(arena_bytes),
                                       int(max_active), C.c_void_p(self.stream)),
               "server_create", False)
        self.h = h
        self.live = {}   # rid -> tensors the library points into

    @staticmethod
    def request_bytes(n: int, m: int, d: int) -> int:
        return int(lib().pot_server_request_bytes(n, m, d))

    @staticmethod
    def arena_overhead(max_active: int) -> int:
        return int(lib().pot_server_arena_overhead(max_active))

    def submit(self, X, Y, K: int, *, want_TX: bool = True, **kw):
        """Returns a request id, or None when it cannot be admitted now."""
        torch = _torch()
        _dev_f32(X, "X")
        _dev_f32(Y, "Y")
        n, d = X.shape
        m = Y.shape[0]
        p, keep = _params(K, **kw)
        f = torch.empty(n, dtype=torch.float32, device=X.device)
        G = torch.empty((K, m), dtype=torch.float32, device=X.device)
        TX = torch.empty((n, d), dtype=torch.float32, device=X.device) if want_TX else None
        rid = C.c_int64()
        st = lib().pot_server_submit(self.h, _ptr(X), n, _ptr(Y), m, d, C.byref(p), _ptr(f),
                                     _ptr(G), _ptr(TX), C.byref(rid))
        if st == POT_BUSY:
            return None
        _check(st, "server_submit", False)
        self.live[rid.value] = (X, Y, f, G, TX, keep)
        return rid.value

    def step(self):
        """One tick; returns (n_active, n_finished_in_this_tick)."""
        a, fin = C.c_int32(), C.c_int32()
        _check(lib().pot_server_step(self.h, C.byref(a), C.byref(fin)), "server_step", False)
        return a.value, fin.value

    def poll(self, rid: int):
        """None while in flight, else (f, G, TX, ProgOTInfo); raises PotError
        with the request's status when it failed."""
        info = pot_progot_info()
        st = lib().pot_server_poll(self.h, int(rid), C.byref(info))
        if st == POT_BUSY:
            return None
        # the request is finished (or unknown): drop its tensors before a
        # failure status raises
        entry = self.live.pop(rid, None)
        _check(st, "server_poll")
        _, _, f, G, TX, _ = entry
        return f, G, TX, _info(info, st)

    def close(self):
        if getattr(self, "h", None):
            lib().pot_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def timing_enable(on: bool = True, every: int = 1) -> None:
    """Start (and clear) or stop the library's per-launch kernel timing;
    while on, launches 0, every, 2 every, ... of each timed kernel are
    timed."""
    if on and every < 1:
        raise ValueError("every must be >= 1")
    _check(lib().pot_timing_enable(int(every) if on else 0), "timing_enable", False)


def timing_read():
    """(lse_ms, lse_launches, map_ms, map_launches) summed over the timed
    launches; waits for the recorded events."""
    a, b = C.c_double(), C.c_int64()
    c, d = C.c_double(), C.c_int64()
    _check(lib().pot_timing_read(C.byref(a), C.byref(b), C.byref(c), C.byref(d)), "timing_read",
           False)
    return a.value, b.value, c.value, d.value


def to_device(a: np.ndarray, device="cuda"):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
