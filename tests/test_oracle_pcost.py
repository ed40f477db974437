"""Pins of the oracle's general-cost path, h = (1/p)|.|_p^p.

Each pin checks the oracle against something other than its own formulas:
exact values, the calculus identities that tie h, grad h, h* and grad h*
together, the independently pinned squared-Euclidean oracle (p = 2 is half
that cost), finite differences of the entropic potential, and exact optimal
assignments from a library solver and from sorting as eps -> 0.
"""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from oracle import pcost
from oracle.sinkhorn import cost_matrix, sinkhorn
import workloads


def test_h_exact_values():
    """|1|^1.5 + |-4|^1.5 + |1/4|^1.5 = 1 + 8 + 1/8; h = that / 1.5."""
    z = np.array([1.0, -4.0, 0.25])
    assert pcost.h_p(z, 1.5) == pytest.approx(9.125 / 1.5, rel=1e-15)
    assert pcost.h_p(z, 2.0) == pytest.approx((1 + 16 + 1 / 16) / 2, rel=1e-15)
    assert pcost.h_p(np.zeros(5), 1.5) == 0.0
    np.testing.assert_array_equal(pcost.grad_h(np.array([4.0, -9.0, 0.0]), 1.5), [2.0, -3.0, 0.0])
    np.testing.assert_array_equal(pcost.grad_h_star(np.array([2.0, -3.0, 0.0]), 1.5), [4.0, -9.0, 0.0])


def test_cost_matrix_p2_is_half_squared():
    X, Y = workloads.gmm(seed=21, n=37, m=29, d=6)
    np.testing.assert_allclose(pcost.cost_matrix_p(X, Y, 2.0), 0.5 * cost_matrix(X, Y),
                               rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("p", [1.25, 1.5, 3.0])
def test_grad_h_finite_difference(p):
    """grad h is the gradient of h (central differences, away from 0)."""
    rng = np.random.default_rng(5)
    z = rng.uniform(0.3, 2.0, size=7) * rng.choice([-1.0, 1.0], size=7)
    g = pcost.grad_h(z, p)
    hs = 1e-6
    for k in range(7):
        e = np.zeros(7)
        e[k] = hs
        fd = (pcost.h_p(z + e, p) - pcost.h_p(z - e, p)) / (2 * hs)
        assert fd == pytest.approx(g[k], rel=1e-8, abs=1e-9)


@pytest.mark.parametrize("p", [1.25, 1.5, 3.0])
def test_conjugate_identities(p):
    """grad h* inverts grad h, and Fenchel-Young holds with equality at
    w = grad h(z): h(z) + h*(w) = <z, w>; elsewhere it is an inequality."""
    rng = np.random.default_rng(6)
    Z = rng.standard_normal((50, 9)) * 2.0
    W = pcost.grad_h(Z, p)
    np.testing.assert_allclose(pcost.grad_h_star(W, p), Z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pcost.h_p(Z, p) + pcost.h_star(W, p), (Z * W).sum(1), rtol=1e-12)
    W2 = W + rng.standard_normal(W.shape) * 0.3
    assert np.all(pcost.h_p(Z, p) + pcost.h_star(W2, p) >= (Z * W2).sum(1) - 1e-12)


def test_map_p2_equals_squared_map():
    """p = 2: T for |.|^2/2 at eps with g equals the squared-Euclidean map at
    2 eps with 2 g (independent oracle code)."""
    X, Y = workloads.gmm(seed=22, n=40, m=33, d=5)
    g = np.random.default_rng(3).standard_normal(33)
    eps = 3.0
    for alpha in (1.0, 0.4):
        np.testing.assert_allclose(pcost.entropic_map_p(X, Y, g, eps, 2.0, alpha=alpha),
                                   oracle.entropic_map(X, Y, 2 * g, 2 * eps, alpha=alpha),
                                   rtol=1e-12, atol=1e-12)


def test_sinkhorn_p2_equals_squared_at_twice_eps():
    X, Y = workloads.gmm(seed=23, n=50, m=41, d=4)
    a, b = workloads.weights(50, seed=1), workloads.weights(41, seed=2)
    C = cost_matrix(X, Y)
    eps = 0.05 * C.mean()
    r2 = sinkhorn(a, X, b, Y, eps, 0.0, n_iter=30, C=C)
    rp = sinkhorn(a, X, b, Y, eps / 2, 0.0, n_iter=30, C=pcost.cost_matrix_p(X, Y, 2.0))
    np.testing.assert_allclose(rp.f, r2.f / 2, rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(rp.g, r2.g / 2, rtol=1e-11, atol=1e-11)


def test_progot_p2_matches_squared_progot():
    """The eps rule is relative to the mean cost, so ProgOT with |.|^2/2 runs
    at half the eps of the squared-Euclidean ProgOT on the same problem: the
    iterates X^(k) coincide and the potentials are halved."""
    X, Y = workloads.c1(seed=3, n=60, m=60, d=3)
    a = b = np.full(60, 1 / 60)
    rs = oracle.progot(a, X, b, Y, 3, theta=1.0, n_iter=40)
    rp = pcost.progot_p(a, X, b, Y, 3, 2.0, theta=1.0, n_iter=40)
    np.testing.assert_allclose(rp.eps, rs.eps / 2, rtol=1e-13)
    np.testing.assert_allclose(rp.G, rs.G / 2, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(rp.TX, rs.TX, rtol=1e-10, atol=1e-10)
    Q = workloads.c1_holdout(seed=3, n=60, d=3, m_test=25)
    np.testing.assert_allclose(pcost.progot_map_p(Q, Y, rp.G, rp.eps, rp.alpha, 2.0),
                               oracle.progot_map(Q, Y, rs.G, rs.eps, rs.alpha),
                               rtol=1e-10, atol=1e-10)


@pytest.mark.parametrize("p", [1.5, 3.0])
def test_map_is_x_minus_grad_h_star_of_potential_gradient(p):
    """eq. Tent: T(x) = x - grad h*(grad f(x)) with f the entropic potential
    of eq. entpot; grad f taken here by central differences of f."""
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((30, 4))
    g = rng.standard_normal(30) * 0.3
    Xq = rng.standard_normal((5, 4)) * 0.8
    eps = 0.7
    hs = 1e-5
    Gf = np.zeros_like(Xq)
    for k in range(4):
        e = np.zeros(4)
        e[k] = hs
        Gf[:, k] = (pcost.potential_p(Xq + e, Y, g, eps, p)
                    - pcost.potential_p(Xq - e, Y, g, eps, p)) / (2 * hs)
    np.testing.assert_allclose(pcost.entropic_map_p(Xq, Y, g, eps, p),
                               Xq - pcost.grad_h_star(Gf, p), rtol=1e-6, atol=1e-6)


def test_translation_equivariance():
    X, Y = workloads.gmm(seed=24, n=20, m=25, d=3)
    g = np.random.default_rng(8).standard_normal(25)
    t = np.array([0.75, -1.5, 2.0])
    np.testing.assert_allclose(pcost.entropic_map_p(X + t, Y + t, g, 2.0, 1.5),
                               pcost.entropic_map_p(X, Y, g, 2.0, 1.5) + t, rtol=1e-10, atol=1e-10)


def _small_eps_fit(X, Y, p, frac):
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    C = pcost.cost_matrix_p(X, Y, p)
    eps = frac * C.mean()
    r = sinkhorn(a, X, a, Y, eps, 1e-5, max_iter=200_000, C=C)
    assert r.converged
    return C, r, eps


@pytest.mark.parametrize("p", [1.5, 3.0])
def test_small_eps_recovers_exact_assignment(p):
    """As eps -> 0 the coupling tends to the optimal permutation / n (a
    library assignment solver on the same cost) and the map sends x_i to
    its partner y_sigma(i)."""
    rng = np.random.default_rng(9)
    X, Y = rng.standard_normal((7, 3)), rng.standard_normal((7, 3)) + 0.5
    C, r, eps = _small_eps_fit(X, Y, p, 5e-4)
    rows, cols = linear_sum_assignment(C)
    P = oracle.coupling(r.f, r.g, C, eps)
    np.testing.assert_allclose(P[rows, cols] * 7, 1.0, atol=1e-3)
    T = pcost.entropic_map_p(X, Y, r.g, eps, p)
    np.testing.assert_allclose(T[rows], Y[cols], atol=1e-3)


def test_small_eps_one_dimension_is_monotone():
    """d = 1: for a strictly convex h the optimal matching is the sorted one."""
    rng = np.random.default_rng(10)
    x, y = rng.uniform(-2, 2, 9), rng.uniform(-1, 3, 9)
    X, Y = x[:, None], y[:, None]
    _, r, eps = _small_eps_fit(X, Y, 1.5, 2e-4)
    T = pcost.entropic_map_p(X, Y, r.g, eps, 1.5)[:, 0]
    np.testing.assert_allclose(T[np.argsort(x)], np.sort(y), atol=1e-3)


def test_large_eps_product_coupling():
    """eps >> cost: P tends to a b^T, and the map to the b-weighted mean
    pushed through grad h* of the mean gradient, which for y_j symmetric
    about x is x itself."""
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((6, 2))
    Y = np.concatenate([Y, -Y])                                # symmetric about 0
    a = np.full(12, 1 / 12)
    C = pcost.cost_matrix_p(np.zeros((12, 2)), Y, 1.5)
    r = sinkhorn(a, np.zeros((12, 2)), a, Y, 1e6, 1e-12, max_iter=50, C=C)
    np.testing.assert_allclose(oracle.coupling(r.f, r.g, C, 1e6), np.full((12, 12), 1 / 144),
                               rtol=1e-5)
    np.testing.assert_allclose(pcost.entropic_map_p(np.zeros((1, 2)), Y, r.g, 1e6, 1.5),
                               np.zeros((1, 2)), atol=1e-6)


def test_progot_p_k1_is_one_solve_and_map():
    X, Y = workloads.gmm(seed=25, n=30, m=30, d=3)
    a = np.full(30, 1 / 30)
    r = pcost.progot_p(a, X, a, Y, 1, 1.5, theta=1.0, n_iter=25)
    C = pcost.cost_matrix_p(X, Y, 1.5)
    eps = C.mean() / 20
    s = sinkhorn(a, X, a, Y, eps, 0.0, n_iter=25, C=C)
    assert r.eps[0] == pytest.approx(eps, rel=1e-15)
    np.testing.assert_allclose(r.G[0], s.g, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(r.TX, pcost.entropic_map_p(X, Y, s.g, eps, 1.5), rtol=1e-13)


def test_eps_scheduler_p2_is_half_squared():
    """Alg. 4 with |.|^2/2: eps_0, sigma and every grid eps halve, the maps
    and hence the hold-out scores and the selected scale are unchanged, and
    the schedule halves."""
    X, Y = workloads.c1(seed=2, n=80, m=70, d=3)
    Yt = workloads.c1_holdout(seed=2, n=80, d=3, m_test=40)
    a, b = np.full(80, 1 / 80), np.full(70, 1 / 70)
    alpha = oracle.schedules.alpha_schedule(4)
    rs, ins = oracle.schedules.eps_scheduler(a, X, b, Y, alpha, Yt, tau=1e-9)
    rp, inp = oracle.schedules.eps_scheduler(a, X, b, Y, alpha, Yt, tau=1e-9, cost_p=2.0)
    assert inp["p_star"] == ins["p_star"]
    np.testing.assert_allclose(inp["errors"], ins["errors"], rtol=1e-7)
    np.testing.assert_allclose(rp, rs / 2, rtol=1e-12)
