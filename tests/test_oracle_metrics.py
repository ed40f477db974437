"""Pins of the oracle's evaluation metrics (Sinkhorn divergence, <P, C>,
sum P log P, trace / KL of the coupling-recovery benchmark) against what
the mathematics fixes."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from oracle.sinkhorn import cost_matrix
import workloads


def _cloud(seed=3, n=60, d=3):
    return workloads.gmm(seed=seed, n=n, m=n, d=d, n_comp=2)[0]


def test_divergence_of_a_cloud_with_itself_is_zero():
    X = _cloud()
    a = np.full(X.shape[0], 1.0 / X.shape[0])
    D, oxy, oxx, oyy, _ = metrics.sinkhorn_divergence(a, X, a, X, tau=1e-10)
    assert abs(D) < 1e-10 * abs(oxy)


def test_divergence_translation_identity():
    """Y = X + t with equal uniform weights: C(X, Y)_ij = C(X, X)_ij
    - 2<x_i, t> + 2<x_j, t> + |t|^2.  The middle terms are separable, so the
    potentials absorb them and the coupling is that of (X, X); the objective
    rises by |t|^2 exactly (the separable terms integrate to zero against
    equal marginals), while OT(Y, Y) = OT(X, X).  Hence D_eps(X, X + t) =
    |t|^2 for every eps."""
    # points on a 2^-10 grid and a short t: X + t is exact in FP32
    X = (np.round(_cloud(seed=5, n=50, d=3) * 1024) / 1024).astype(np.float32)
    t = np.array([0.75, -1.125, 0.375], dtype=np.float32)
    Y = (X + t).astype(np.float32)
    assert np.array_equal(Y.astype(np.float64) - X.astype(np.float64), np.tile(t.astype(np.float64), (50, 1)))
    tt = float((t.astype(np.float64) ** 2).sum())
    a = np.full(X.shape[0], 1.0 / X.shape[0])
    mc = oracle.mean_cost(X, X)
    # eps where Alg. 1 reaches 1e-12 on this clustered cloud (at a few
    # percent of the mean cost it needs > 2e4 iterations, as textbook
    # Sinkhorn-Knopp scaling does too)
    for eps in (0.5 * mc, 2.0 * mc):
        D, *_ = metrics.sinkhorn_divergence(a, X, a, Y, eps=eps, tau=1e-12)
        assert abs(D - tt) < 1e-9 * tt, (eps, D, tt)


def test_divergence_large_eps_limit():
    """As eps -> infinity the coupling tends to a (x) b and D tends to
    mean C(X, Y) - (mean C(X, X) + mean C(Y, Y))/2 = |xbar - ybar|^2; the
    gap shrinks like 1/eps (ratio ~10 per decade)."""
    X = _cloud(seed=7, n=40, d=2)
    Y = workloads.gmm(seed=8, n=40, m=40, d=2, n_comp=2)[1]
    a = np.full(40, 1.0 / 40)
    lim = float(((X.astype(np.float64).mean(0) - Y.astype(np.float64).mean(0)) ** 2).sum())
    mc = oracle.mean_cost(X, Y)
    gaps = []
    for eps in (100 * mc, 1000 * mc):
        D, *_ = metrics.sinkhorn_divergence(a, X, a, Y, eps=eps, tau=1e-13)
        gaps.append(abs(D - lim))
    assert 5 < gaps[0] / gaps[1] < 20


def test_primal_parts_match_the_dual():
    """At convergence <P, C> + eps (sum P log P - sum P) equals the objective
    of eq. entdual (strong duality), tying the two new sums to the dual."""
    X, Y = workloads.gmm(seed=9, n=70, m=50, d=3)
    a, b = np.full(70, 1 / 70), np.full(50, 1 / 50)
    C = cost_matrix(X, Y)
    eps = 0.05 * C.mean()
    r = oracle.sinkhorn(a, X, b, Y, eps, 1e-12, max_iter=100_000, C=C)
    P = oracle.coupling(r.f, r.g, C, eps)
    primal = metrics.transport_cost(P, C) + eps * (metrics.p_log_p(P) - P.sum())
    dual = oracle.dual_objective(r.f, r.g, C, eps, a, b)
    assert abs(primal - dual) < 1e-9 * abs(dual)


def test_diag_metrics_limits():
    """Product coupling (eps -> infinity): Tr P = 1/n, KL(I/n || P) = log n.
    Identity recovery (Y = X G^T, G SPD, small eps): Tr P -> 1, KL -> 0."""
    n = 64
    P = np.full((n, n), 1.0 / n ** 2)
    tr, kl = metrics.diag_metrics(P)
    assert abs(tr - 1 / n) < 1e-15 and abs(kl - np.log(n)) < 1e-12
    X, Y = workloads.spd_pair(seed=9, n=128, d=6)
    a = np.full(128, 1 / 128)
    C = cost_matrix(X, Y)
    r = oracle.sinkhorn(a, X, a, Y, 0.1 * C.mean() / 20, 1e-6, max_iter=100_000, C=C)
    tr, kl = metrics.diag_metrics(oracle.coupling(r.f, r.g, C, 0.1 * C.mean() / 20))
    assert tr > 0.99 and 0 <= kl < 0.02


def test_divergence_general_cost_p2_is_half_squared():
    """h = |.|^2/2: every OT_eps value is half the squared-Euclidean one at
    twice eps (the same coupling), and the default eps_D halves with the
    mean cost, so D_h = D/2 with both defaults."""
    X, Y = workloads.gmm(seed=61, n=40, m=30, d=3)
    a, b = np.full(40, 1 / 40), np.full(30, 1 / 30)
    ds = metrics.sinkhorn_divergence(a, X, b, Y, tau=1e-10)
    dp = metrics.sinkhorn_divergence(a, X, b, Y, tau=1e-10, cost_p=2.0)
    assert dp[4] == pytest.approx(ds[4] / 2, rel=1e-12)
    np.testing.assert_allclose(dp[:4], np.asarray(ds[:4]) / 2, rtol=1e-8, atol=1e-10)


def test_divergence_general_cost_separates():
    """p = 1.5: exp(-h/eps) is a positive-definite kernel (p <= 2), so the
    divergence vanishes on equal clouds and is positive otherwise, growing
    with a translation."""
    X = workloads.gmm(seed=62, n=20, m=4, d=2)[0]
    a = np.full(20, 1 / 20)
    eps = 4 * metrics.eps_divergence_default(X, cost_p=1.5)
    assert abs(metrics.sinkhorn_divergence(a, X, a, X, eps=eps, tau=1e-10, cost_p=1.5)[0]) < 1e-9
    vals = [metrics.sinkhorn_divergence(a, X, a, X + s, eps=eps, tau=1e-10, cost_p=1.5)[0]
            for s in (0.25, 1.0)]
    assert 0 < vals[0] < vals[1]
