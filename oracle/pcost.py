"""General translation-invariant costs h = (1/p)|.|_p^p (oracle).

Test infrastructure only.

Sec. 3 states ProgOT for any strictly convex translation-invariant cost
h(x - y); the experiments of Sec. 5.2 (coupling solver) and the appendix on
map estimation use h(z) = (1/p) sum_k |z_k|^p with p = 1.5.  For this h:

* grad h(z)_k = sign(z_k) |z_k|^(p-1);
* its convex conjugate is h*(w) = (1/q) sum_k |w_k|^q with 1/p + 1/q = 1,
  so grad h*(w)_k = sign(w_k) |w_k|^(q-1) = sign(w_k) |w_k|^(1/(p-1)),
  the inverse map of grad h;
* the entropic map (eq. Tent) is T(x) = x - grad h*(grad f_eps(x)) with
  grad f_eps(x) = sum_j p_j(x) grad h(x - y_j),
  p_j(x) = softmax_j((g_j - h(x - y_j))/eps);
* Alg. 2 moves the source by X <- X - alpha_k Z with
  Z_i = grad h*(sum_j Q_ij grad h(x_i - y_j)), Q = diag(1/P 1) P, which at a
  training point is alpha_k (x_i - T(x_i)): the same McCann-type step;
* Alg. 3 applies y <- y - alpha_k grad h*(p^T Delta), Delta_j = grad h(y - y_j),
  the same map at an arbitrary point.

The potentials use the convention of the squared-Euclidean path
(P_ij = exp((f_i + g_j - C_ij)/eps)), so Alg. 1 runs unchanged on the cost
matrix C_ij = h(x_i - y_j) (``sinkhorn(..., C=cost_matrix_p(X, Y, p))``), and
eps_k = theta * mean(C)/20 per step (App. C: the scaled average of the cost
h over all pairs).

With p = 2, h = |.|^2/2 is half the squared-Euclidean cost, so every result
here equals the squared-Euclidean one at twice eps with potentials halved;
the tests use that as one of the pins.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import schedules
from .sinkhorn import sinkhorn, marginal_errors, _run, _CHUNK


def _f64(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64)


def h_p(Z, p: float) -> np.ndarray:
    """h(z) = (1/p) sum_k |z_k|^p over the last axis."""
    return (np.abs(_f64(Z)) ** p).sum(axis=-1) / p


def grad_h(Z, p: float) -> np.ndarray:
    """grad h(z)_k = sign(z_k) |z_k|^(p-1)."""
    Z = _f64(Z)
    return np.sign(Z) * np.abs(Z) ** (p - 1.0)


def h_star(W, p: float) -> np.ndarray:
    """h*(w) = (1/q) sum_k |w_k|^q, q = p/(p-1)."""
    q = p / (p - 1.0)
    return (np.abs(_f64(W)) ** q).sum(axis=-1) / q


def grad_h_star(W, p: float) -> np.ndarray:
    """grad h*(w)_k = sign(w_k) |w_k|^(1/(p-1))."""
    W = _f64(W)
    return np.sign(W) * np.abs(W) ** (1.0 / (p - 1.0))


def cost_matrix_p(X, Y, p: float) -> np.ndarray:
    """C_ij = h(x_i - y_j), by direct differences."""
    X, Y = _f64(X), _f64(Y)
    n, m = X.shape[0], Y.shape[0]
    C = np.empty((n, m))

    def work(lo, hi):
        C[lo:hi] = h_p(X[lo:hi, None, :] - Y[None, :, :], p)

    step = max(1, min(_CHUNK, (1 << 23) // max(1, m * X.shape[1])))
    _run(work, n, step)
    return C


def map_weights_p(Xq, Y, g, eps, p: float) -> np.ndarray:
    """Row-stochastic p_ij = softmax_j((g_j - h(x_i - y_j))/eps)."""
    S = (_f64(g)[None, :] - cost_matrix_p(Xq, Y, p)) / eps
    S -= S.max(axis=1, keepdims=True)
    P = np.exp(S)
    P /= P.sum(axis=1, keepdims=True)
    return P


def potential_p(Xq, Y, g, eps, p: float, b=None) -> np.ndarray:
    """The entropic potential at arbitrary points (eq. entpot, with the
    potentials' convention above): f(x) = -eps log sum_j exp((g_j -
    h(x - y_j))/eps), up to the additive constant eps log a that the map
    does not see.  ``b`` (optional) adds eps log b_j inside, the convention
    where the weights sit outside the potentials."""
    S = (_f64(g)[None, :] - cost_matrix_p(Xq, Y, p)) / eps
    if b is not None:
        S = S + np.log(_f64(b))[None, :]
    mx = S.max(axis=1)
    return -eps * (mx + np.log(np.exp(S - mx[:, None]).sum(axis=1)))


def entropic_map_p(Xq, Y, g, eps, p: float, alpha: float = 1.0) -> np.ndarray:
    """x - alpha grad h*(sum_j p_j(x) grad h(x - y_j)) for every row x of Xq
    (eq. Tent for h; alpha = 1 gives T(x), alpha < 1 the step of Alg. 2/3)."""
    Xq, Y = _f64(Xq), _f64(Y)
    out = np.empty_like(Xq)
    step = max(1, (1 << 21) // max(1, Y.shape[0] * Y.shape[1]))
    for lo in range(0, Xq.shape[0], step):
        hi = min(Xq.shape[0], lo + step)
        W = map_weights_p(Xq[lo:hi], Y, g, eps, p)
        D = grad_h(Xq[lo:hi, None, :] - Y[None, :, :], p)       # (q, m, d)
        Gf = np.einsum("qj,qjd->qd", W, D)                        # grad f_eps(x)
        out[lo:hi] = Xq[lo:hi] - alpha * grad_h_star(Gf, p)
    return out


@dataclass
class ProgOTpResult:
    f: np.ndarray
    G: np.ndarray
    eps: np.ndarray
    alpha: np.ndarray
    iters: list = field(default_factory=list)
    errs: list = field(default_factory=list)
    X_last: np.ndarray = None
    TX: np.ndarray = None
    mean_cost: list = field(default_factory=list)
    final_row_err: float = 0.0
    final_col_err: float = 0.0


def progot_p(a, X, b, Y, K: int, p: float, *, alpha_kind: str = "constant", eps=None,
             theta: float = 1.0, tau=1e-3, max_iter: int = 10_000, n_iter=None) -> ProgOTpResult:
    """Alg. 2 for the cost h: K warm-started Sinkhorn solves on C(X^(k), Y),
    each followed by X^(k+1) = X^(k) - alpha_k Z (warm start (1 - alpha_k),
    as printed).  eps: None for eps_k = theta * mean C(X^(k), Y)/20, or an
    explicit schedule.  n_iter: None (stop on tau), one count for every
    solve, or one count per solve."""
    alpha = schedules.alpha_schedule(K, alpha_kind)
    taus = np.broadcast_to(np.asarray(tau, dtype=np.float64), (K,))
    Xk = _f64(X).copy()
    Yd = _f64(Y)
    n, m = Xk.shape[0], Yd.shape[0]
    f, g_prev = np.zeros(n), np.zeros(m)
    G = np.zeros((K, m))
    eps_used = np.zeros(K)
    out = ProgOTpResult(f=f, G=G, eps=eps_used, alpha=alpha)
    its = [n_iter] * K if n_iter is None or np.isscalar(n_iter) else list(n_iter)
    for k in range(K):
        C = cost_matrix_p(Xk, Yd, p)
        mc = float(C.mean())
        out.mean_cost.append(mc)
        eps_k = float(theta * mc / 20.0) if eps is None else float(eps[k])
        eps_used[k] = eps_k
        w = alpha[k]
        res = sinkhorn(a, Xk, b, Yd, eps_k, float(taus[k]), (1.0 - w) * f, (1.0 - w) * g_prev,
                       max_iter=max_iter, n_iter=its[k], C=C)
        f = res.f
        G[k] = res.g
        g_prev = res.g
        out.iters.append(res.iters)
        out.errs.append(res.err)
        out.X_last = Xk
        Xk = entropic_map_p(Xk, Yd, res.g, eps_k, p, alpha=alpha[k])
        if k == K - 1:
            out.final_row_err, out.final_col_err = marginal_errors(res.f, res.g, C, eps_k, a, b)
    out.f = f
    out.TX = Xk
    return out


def progot_map_p(Xq, Y, G, eps, alpha, p: float) -> np.ndarray:
    """Alg. 3 for the cost h: y <- x, then y <- y - alpha_k grad h*(sum_j
    p_j grad h(y - y_j)) for k = 0..K-1, the last alpha reset to 1."""
    alpha = np.asarray(alpha, dtype=np.float64).copy()
    alpha[-1] = 1.0
    y = _f64(Xq).copy()
    for k in range(len(alpha)):
        y = entropic_map_p(y, Y, G[k], float(eps[k]), p, alpha=float(alpha[k]))
    return y
