"""Evaluation metrics of couplings and clouds (oracle).

Test infrastructure only.

* OT_eps(X, Y): the objective of eq. entdual at Alg. 1's solution,
  <f, a> + <g, b> - eps sum_ij P_ij.
* Sinkhorn divergence (eq. sink_div):
  D(X, Y) = OT_eps(X, Y) - (OT_eps(X, X) + OT_eps(Y, Y)) / 2, with the default
  eps_D = 5 % of the mean cost within the target cloud (App. on experiment
  details); with the squared-Euclidean cost, or with h = (1/p)|.|_p^p as in
  the map appendix's tables for the 1.5-norm cost.
* <P, C> and sum P log P of a coupling.
* Coupling-recovery metrics of Sec. 5.3 for n = m, where the true coupling
  is the identity / n: the trace Tr P and KL(I/n || P), read as
  -log n - (1/n) sum_i log P_ii (the printed "-n sum" cannot be the KL of
  two couplings with marginals 1/n).
"""
from __future__ import annotations

import numpy as np

from .sinkhorn import cost_matrix, dual_objective, sinkhorn
from .pcost import cost_matrix_p


def transport_cost(P, C) -> float:
    """<P, C> = sum_ij P_ij C_ij."""
    return float((np.asarray(P, np.float64) * C).sum())


def p_log_p(P) -> float:
    """sum_ij P_ij log P_ij (0 log 0 = 0)."""
    P = np.asarray(P, np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        return float(np.where(P > 0, P * np.log(P), 0.0).sum())


def _cost(X, Y, cost_p):
    return cost_matrix(X, Y) if cost_p is None else cost_matrix_p(X, Y, cost_p)


def eps_divergence_default(Y, cost_p=None) -> float:
    """5 % of the mean pairwise cost within Y."""
    return float(0.05 * _cost(Y, Y, cost_p).mean())


def ot_value(a, X, b, Y, eps, tau, max_iter=100_000, cost_p=None) -> float:
    """OT_eps(X, Y): objective of eq. entdual at Alg. 1's solution to tau
    (cost |.|^2, or h = (1/p)|.|_p^p with cost_p = p)."""
    C = _cost(X, Y, cost_p)
    r = sinkhorn(a, X, b, Y, eps, tau, max_iter=max_iter, C=C)
    return dual_objective(r.f, r.g, C, eps, a, b)


def sinkhorn_divergence(a, X, b, Y, eps=None, tau=1e-6, max_iter=100_000, cost_p=None):
    """(D, OT(X, Y), OT(X, X), OT(Y, Y), eps) of eq. sink_div; cost_p = p
    evaluates it with h = (1/p)|.|_p^p, as the map appendix's tables do."""
    if eps is None:
        eps = eps_divergence_default(Y, cost_p)
    oxy = ot_value(a, X, b, Y, eps, tau, max_iter, cost_p)
    oxx = ot_value(a, X, a, X, eps, tau, max_iter, cost_p)
    oyy = ot_value(b, Y, b, Y, eps, tau, max_iter, cost_p)
    return oxy - 0.5 * (oxx + oyy), oxy, oxx, oyy, eps


def diag_metrics(P):
    """(Tr P, KL(I/n || P)) = (sum_i P_ii, -log n - (1/n) sum_i log P_ii)."""
    P = np.asarray(P, np.float64)
    n = P.shape[0]
    d = np.diag(P)
    return float(d.sum()), float(-np.log(n) - np.log(d).sum() / n)
