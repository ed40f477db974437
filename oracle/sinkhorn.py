"""Log-domain Sinkhorn on a materialised cost matrix, FP64 (oracle).

Test infrastructure only; see the package docstring for the readings of the
paper adopted here.

Follows Alg. 1 (Sinkhorn) of Sec. 2 and the entropic dual (eq. entdual):
for eps > 0 the entropic coupling is P = exp((f (+) g - C)/eps) where (f, g)
maximise <f, a> + <g, b> - eps <e^{f/eps}, K e^{g/eps}> with K = e^{-C/eps}.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

THREADS = os.cpu_count() or 1
_POOL: ThreadPoolExecutor | None = None
_CHUNK = 256


def _pool() -> ThreadPoolExecutor:
    global _POOL
    if _POOL is None:
        _POOL = ThreadPoolExecutor(THREADS)
    return _POOL


def _chunks(n: int, step: int = _CHUNK):
    return [(s, min(n, s + step)) for s in range(0, n, step)]


def _run(work, n: int, step: int = _CHUNK):
    """Apply work(lo, hi) over row chunks; threads only when there are
    several chunks."""
    ch = _chunks(n, step)
    if len(ch) == 1:
        work(*ch[0])
    else:
        list(_pool().map(lambda r: work(*r), ch))


def _f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def cost_matrix(X, Y) -> np.ndarray:
    """C_ij = h(x_i - y_j) with h = |.|^2, by direct differences (Alg. 1,
    the cost line; squared-Euclidean cost of Sec. 5)."""
    X, Y = _f64(X), _f64(Y)
    n, m = X.shape[0], Y.shape[0]
    C = np.empty((n, m))

    def work(lo, hi):
        D = X[lo:hi, None, :] - Y[None, :, :]
        C[lo:hi] = np.einsum("ijk,ijk->ij", D, D)

    step = max(1, min(_CHUNK, (1 << 24) // max(1, m * X.shape[1])))
    _run(work, n, step)
    return C


def mean_cost(X, Y) -> float:
    """(1/nm) sum_ij h(x_i - y_j): the scale behind eps_0 (Alg. 4, first set
    line) and the per-step mean cost of the coupling experiments (App. C)."""
    return float(cost_matrix(X, Y).mean())


def softmin_rows(C: np.ndarray, v: np.ndarray, eps: float) -> np.ndarray:
    """LSE_j((v_j - C_ij)/eps) for each row i; -eps times this is the
    soft-min min_eps(C - v) of Sec. 2 (notation below Alg. 1)."""
    out = np.empty(C.shape[0])

    def work(lo, hi):
        blk = (v[None, :] - C[lo:hi]) / eps
        mx = blk.max(axis=1)
        out[lo:hi] = mx + np.log(np.exp(blk - mx[:, None]).sum(axis=1))

    _run(work, C.shape[0])
    return out


def softmin_cols(C: np.ndarray, u: np.ndarray, eps: float) -> np.ndarray:
    """LSE_i((u_i - C_ij)/eps) for each column j."""
    out = np.empty(C.shape[1])

    def work(lo, hi):
        blk = (u[:, None] - C[:, lo:hi]) / eps
        mx = blk.max(axis=0)
        out[lo:hi] = mx + np.log(np.exp(blk - mx[None, :]).sum(axis=0))

    _run(work, C.shape[1])
    return out


def _row_sums(f, g, C, eps) -> np.ndarray:
    out = np.empty(C.shape[0])

    def work(lo, hi):
        out[lo:hi] = np.exp((f[lo:hi, None] + g[None, :] - C[lo:hi]) / eps).sum(axis=1)

    _run(work, C.shape[0])
    return out


def _col_sums(f, g, C, eps) -> np.ndarray:
    out = np.empty(C.shape[1])

    def work(lo, hi):
        out[lo:hi] = np.exp((f[:, None] + g[None, lo:hi] - C[:, lo:hi]) / eps).sum(axis=0)

    _run(work, C.shape[1])
    return out


def coupling(f, g, C, eps) -> np.ndarray:
    """P_ij = exp((f_i + g_j - C_ij)/eps) (Alg. 1, returned coupling)."""
    return np.exp((_f64(f)[:, None] + _f64(g)[None, :] - C) / eps)


def marginal_errors(f, g, C, eps, a, b):
    """(|P 1_m - a|_1, |P^T 1_n - b|_1), the marginal criterion (iii) of the
    coupling experiments (Sec. 5.2)."""
    f, g, a, b = _f64(f), _f64(g), _f64(a), _f64(b)
    return (float(np.abs(_row_sums(f, g, C, eps) - a).sum()),
            float(np.abs(_col_sums(f, g, C, eps) - b).sum()))


def dual_objective(f, g, C, eps, a, b) -> float:
    """<f, a> + <g, b> - eps sum_ij P_ij (eq. entdual)."""
    f, g = _f64(f), _f64(g)
    return float(f @ _f64(a) + g @ _f64(b) - eps * _row_sums(f, g, C, eps).sum())


def primal_objective(P, C, eps) -> float:
    """<P, C> + eps sum_ij P_ij (log P_ij - 1), the objective whose dual is
    eq. entdual."""
    with np.errstate(divide="ignore", invalid="ignore"):
        ent = np.where(P > 0, P * (np.log(P) - 1.0), 0.0)
    return float((P * C).sum() + eps * ent.sum())


@dataclass
class SinkhornResult:
    f: np.ndarray
    g: np.ndarray
    iters: int
    err: float          # row-marginal L1 of the returned (f, g)
    converged: bool


def sinkhorn(a, X, b, Y, eps, tau, f_init=None, g_init=None, *, max_iter=10_000,
             n_iter=None, C=None) -> SinkhornResult:
    """Alg. 1, Sink(a, X, b, Y, eps, tau, f_init, g_init).

    Each iteration performs the f-update then the g-update
        f_i <- eps log a_i - eps LSE_j((g_j - C_ij)/eps)
        g_j <- eps log b_j - eps LSE_i((f_i - C_ij)/eps)
    and then evaluates err = |P 1_m - a|_1 for the new (f, g).  It stops as
    soon as err <= tau (``max_iter`` bounds the loop).  With ``n_iter`` set
    exactly that many iterations run and tau is ignored (fixed-iteration
    mode, used to compare potentials iterate by iterate).

    f_init never influences the iterates: the first f-update overwrites f
    (the "+ f" term of Alg. 1 cancels the f inside the soft-min).  It is kept
    for the signature of Alg. 1.
    """
    a, b = _f64(a), _f64(b)
    if C is None:
        C = cost_matrix(X, Y)
    n, m = C.shape
    f = np.zeros(n) if f_init is None else _f64(f_init).copy()
    g = np.zeros(m) if g_init is None else _f64(g_init).copy()
    log_a, log_b = np.log(a), np.log(b)
    limit = n_iter if n_iter is not None else max_iter
    err = float("inf")
    t = 0
    while t < limit:
        t += 1
        f = eps * log_a - eps * softmin_rows(C, g, eps)
        g = eps * log_b - eps * softmin_cols(C, f, eps)
        if n_iter is None or t == limit:
            err = float(np.abs(_row_sums(f, g, C, eps) - a).sum())
            if n_iter is None and err <= tau:
                break
    converged = bool(err <= tau)
    return SinkhornResult(f=f, g=g, iters=t, err=err, converged=converged)
