"""ProgOT (Alg. 2) and the progressive map T_Prog (Alg. 3), FP64 (oracle).

Test infrastructure only.

ProgOT runs K warm-started Sinkhorn solves between the moving source cloud
X^(k) and the fixed target Y; after solve k the source moves along the
McCann-type interpolation X^(k+1) = (1 - alpha_k) X^(k) + alpha_k T_k(X^(k))
(Def. of ProgOT, Sec. 3.1; Alg. 2).  The returned coupling is the one of the
last solve (between X^(K-1) and Y); the fitted map is the list of
(g^(k), eps_k, alpha_k) evaluated by Alg. 3 with the last alpha forced to 1.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .sinkhorn import sinkhorn, cost_matrix, marginal_errors
from .entropic_map import entropic_map
from . import schedules


@dataclass
class ProgOTResult:
    f: np.ndarray                 # potential of the last solve (n)
    G: np.ndarray                 # g^(k), k = 0..K-1 (K x m)
    eps: np.ndarray               # eps_k
    alpha: np.ndarray             # alpha_k (last = 1)
    iters: list = field(default_factory=list)
    errs: list = field(default_factory=list)
    X_last: np.ndarray = None     # X^(K-1): source of the returned coupling
    TX: np.ndarray = None         # X^(K) = T_{K-1}(X^(K-1))
    final_row_err: float = 0.0
    final_col_err: float = 0.0


def progot(a, X, b, Y, K: int, *, alpha_kind: str = "constant", eps=None, theta: float = 1.0,
           tau=1e-3, max_iter: int = 10_000, warm_start: str = "alpha_k",
           n_iter=None) -> ProgOTResult:
    """Alg. 2, ProgOT(a, X, b, Y, (eps_k, alpha_k, tau_k)_k).

    eps: None -> per-step rule eps_k = theta * mean cost(X^(k), Y)/20;
         array -> explicit schedule (e.g. the output of Alg. 4).
    tau: scalar or length-K array.
    warm_start: "alpha_k" (as printed: (1 - alpha_k) f, (1 - alpha_k) g^(k-1))
                or "alpha_prev" ((1 - alpha_{k-1}) instead).
    n_iter: None (stop on tau) or a fixed Sinkhorn iteration count per step.
    """
    alpha = schedules.alpha_schedule(K, alpha_kind)
    taus = np.broadcast_to(np.asarray(tau, dtype=np.float64), (K,))
    Xk = np.asarray(X, dtype=np.float64).copy()
    Yd = np.asarray(Y, dtype=np.float64)
    n, m = Xk.shape[0], Yd.shape[0]
    f = np.zeros(n)
    g_prev = np.zeros(m)
    G = np.zeros((K, m))
    eps_used = np.zeros(K)
    iters, errs = [], []
    res = None
    X_last = Xk
    for k in range(K):
        C = cost_matrix(Xk, Yd)
        eps_k = float(theta * C.mean() / 20.0) if eps is None else float(eps[k])
        eps_used[k] = eps_k
        w = alpha[k] if (warm_start == "alpha_k" or k == 0) else alpha[k - 1]
        res = sinkhorn(a, Xk, b, Yd, eps_k, float(taus[k]), (1.0 - w) * f, (1.0 - w) * g_prev,
                       max_iter=max_iter, n_iter=n_iter, C=C)
        f = res.f
        G[k] = res.g
        g_prev = res.g
        iters.append(res.iters)
        errs.append(res.err)
        X_last = Xk
        Xk = entropic_map(Xk, Yd, res.g, eps_k, alpha=alpha[k])
        if k == K - 1:
            row, col = marginal_errors(res.f, res.g, C, eps_k, a, b)
    return ProgOTResult(f=f, G=G, eps=eps_used, alpha=alpha, iters=iters, errs=errs,
                        X_last=X_last, TX=Xk, final_row_err=row, final_col_err=col)


def progot_map(Xq, Y, G, eps, alpha) -> np.ndarray:
    """Alg. 3, T_Prog[b, Y, (g^(k), eps_k, alpha_k)_k](x) for every row of
    Xq: y <- x, then y <- (1 - alpha_k) y + alpha_k T_k(y) for k = 0..K-1,
    with the last alpha reset to 1."""
    alpha = np.asarray(alpha, dtype=np.float64).copy()
    alpha[-1] = 1.0
    y = np.asarray(Xq, dtype=np.float64).copy()
    for k in range(len(alpha)):
        y = entropic_map(y, Y, G[k], float(eps[k]), alpha=float(alpha[k]))
    return y
