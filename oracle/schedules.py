"""Step-length, regularisation and threshold schedules (oracle).

Test infrastructure only.

alpha: the three schemes of Sec. 4 and the alpha-schedule table (App. C).
K counts Sinkhorn solves, k = 0..K-1.  The table's t-column fixes the
progress after step k (1-based l = k + 1): constant speed t_l = l/K,
accelerated t_l = (l/K)^2, decelerated alpha = 1/e; by convention the last
step is complete (alpha_{K-1} = 1).  alpha_k follows from consecutive
progress values, alpha_k = (t_{k+1} - t_k)/(1 - t_k) with t_0 = 0.

eps: (i) the per-step mean-cost rule of the coupling experiments (App. C),
eps_k = theta * mean_ij h(x_i^(k) - y_j)/20; (ii) Alg. 4 (eps-scheduler).

tau: constant, or decreasing linearly from a loose value (Sec. 4).
"""
from __future__ import annotations

import math

import numpy as np

from .sinkhorn import sinkhorn, cost_matrix
from .entropic_map import entropic_map


def alpha_schedule(K: int, kind: str = "constant") -> np.ndarray:
    if K < 1:
        raise ValueError("K >= 1")
    ell = np.arange(1, K + 1, dtype=np.float64)
    if kind == "constant":
        t = ell / K
    elif kind == "accelerated":
        t = (ell / K) ** 2
    elif kind == "decelerated":
        a = np.full(K, 1.0 / math.e)
        a[-1] = 1.0
        return a
    else:
        raise ValueError(kind)
    t_prev = np.concatenate([[0.0], t[:-1]])
    a = (t - t_prev) / (1.0 - t_prev)
    a[-1] = 1.0
    return a


def progress(alpha) -> np.ndarray:
    """t_k = 1 - prod_{l <= k} (1 - alpha_l): fraction of the path covered
    after step k (Sec. 4, setting step lengths)."""
    return 1.0 - np.cumprod(1.0 - np.asarray(alpha, dtype=np.float64))


def eps_mean_cost(X, Y, theta: float = 1.0) -> float:
    """theta * (1/(20 n m)) sum_ij h(x_i - y_j) (App. C, regularisation for
    the coupling experiments; theta = 1 is the OTT default eps)."""
    return float(theta * cost_matrix(X, Y).mean() / 20.0)


def tau_schedule(K: int, first: float, last: float) -> np.ndarray:
    """Linear decrease from ``first`` to ``last`` over the K solves (Sec. 4,
    setting threshold schedule); first == last gives a constant tau."""
    if K == 1:
        return np.array([last], dtype=np.float64)
    return np.linspace(first, last, K)


def eps_zero(C) -> float:
    """eps_0 of Alg. 4 (its first set line): the mean of the source-target
    cost matrix C over all pairs, divided by 20."""
    return float(np.asarray(C, dtype=np.float64).mean() / 20.0)


def holdout_score(Y_test, TY) -> float:
    """error_p of Alg. 4: sum over the hold-out targets of the squared
    distance |y~ - T(y~)|^2 between each point and its image."""
    D = np.asarray(Y_test, dtype=np.float64) - np.asarray(TY, dtype=np.float64)
    return float((D ** 2).sum())


def eps_scheduler(a, X, b, Y, alpha, Y_test, s_grid=None, beta0: float = 5.0,
                  tau: float = 1e-3, max_iter: int = 10_000, cost_p=None):
    """Alg. 4 (eps-scheduler).

    eps_0 = mean cost between X and Y / 20; sigma = mean intra-target cost
    / 20.  For each s_p, solve Sink(b, Y, b, Y, s_p sigma, tau), map the
    hold-out targets with the one-step entropic map (alpha = 1) and score
    error_p = sum |y~ - T(y~)|^2.  With p* the first argmin, eps_final =
    s_{p*} sigma and the returned schedule is (1 - t'_k) beta0 eps_0 +
    t'_k eps_final with t'_k = 1 - prod_{l=1}^{k} (1 - alpha_l): step 0
    gets beta0 eps_0 and the last step gets eps_final.

    cost_p = p runs it with h = (1/p)|.|_p^p: the mean costs, the grid
    solves and the map use h; the hold-out score stays the squared distance.

    Returns (eps_schedule, info dict).
    """
    if s_grid is None:
        s_grid = [2.0 ** p for p in range(-3, 4)]
    alpha = np.asarray(alpha, dtype=np.float64)
    K = alpha.shape[0]
    if cost_p is None:
        cost, tmap = cost_matrix, entropic_map
    else:
        from . import pcost
        cost = lambda U, V: pcost.cost_matrix_p(U, V, cost_p)
        tmap = lambda Q, V, g, eps, alpha: pcost.entropic_map_p(Q, V, g, eps, cost_p, alpha=alpha)
    eps0 = eps_zero(cost(X, Y))
    Cyy = cost(Y, Y)
    sigma = float(Cyy.mean() / 20.0)
    errors = []
    for s in s_grid:
        eps = s * sigma
        res = sinkhorn(b, Y, b, Y, eps, tau, max_iter=max_iter, C=Cyy)
        Ty = tmap(Y_test, Y, res.g, eps, alpha=1.0)
        errors.append(holdout_score(Y_test, Ty))
    p_star = int(np.argmin(errors))
    eps_final = float(s_grid[p_star] * sigma)
    if K == 1:
        sched = np.array([eps_final])
        tk = np.array([1.0])
    else:
        tk = np.empty(K)
        for k in range(K):
            tk[k] = 1.0 - np.prod(1.0 - alpha[1:k + 1])
        sched = (1.0 - tk) * beta0 * eps0 + tk * eps_final
    return sched, {"eps0": eps0, "sigma": sigma, "errors": errors, "p_star": p_star,
                   "eps_final": eps_final, "t": tk}
