"""Entropic map / barycentric projection and the McCann-type step (oracle).

Test infrastructure only.

For h = |.|^2, h*(z) = |z|^2/4 and grad h*(z) = z/2, so the entropic map of
eq. Tent, T(x) = x - grad h* o grad f_eps(x), reduces to the barycentric
projection T(x) = sum_j p_j(x) y_j with
    p_j(x) = softmax_j((g_j - |x - y_j|^2)/eps).
At a training point x_i, p(x_i) is row i of diag(1/P 1) P (Alg. 2, the
renormalisation line), and Z_i = grad h*(sum_j Q_ij grad h(x_i - y_j))
= x_i - T(x_i), so X <- X - alpha Z is the McCann-type interpolation
S(x) = (1 - alpha) x + alpha T(x) (Def. of ProgOT, Sec. 3.1).
"""
from __future__ import annotations

import numpy as np

from .sinkhorn import cost_matrix


def map_weights(Xq, Y, g, eps) -> np.ndarray:
    """Row-stochastic p_ij = softmax_j((g_j - |x_i - y_j|^2)/eps), FP64."""
    C = cost_matrix(Xq, Y)
    S = (np.asarray(g, dtype=np.float64)[None, :] - C) / eps
    S -= S.max(axis=1, keepdims=True)
    P = np.exp(S)
    P /= P.sum(axis=1, keepdims=True)
    return P


def entropic_map(Xq, Y, g, eps, alpha: float = 1.0) -> np.ndarray:
    """S(x) = (1 - alpha) x + alpha T(x) for every row x of Xq (eq. Tent with
    h = |.|^2; alpha = 1 gives the entropic map itself)."""
    Xq = np.asarray(Xq, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    out = np.empty_like(Xq)
    step = max(1, (1 << 22) // max(1, Y.shape[0]))
    for lo in range(0, Xq.shape[0], step):
        hi = min(Xq.shape[0], lo + step)
        T = map_weights(Xq[lo:hi], Y, g, eps) @ Y
        out[lo:hi] = (1.0 - alpha) * Xq[lo:hi] + alpha * T
    return out
