"""Pins of the FP64 Sinkhorn oracle against what the paper and the mathematics
fix (no GPU).  Each test is chosen so that a plausible mistake in the oracle
(a sign, a dropped factor 2, a transposed operand, a wrong stop rule) fails.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.stats import norm

import oracle
from oracle.sinkhorn import cost_matrix
import workloads


def _small(seed=0, n=60, m=50, d=3, weighted=True):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = (rng.standard_normal((m, d)) * 1.3 + 0.4).astype(np.float32)
    a = workloads.weights(n, seed=seed + 10) if weighted else workloads.weights(n)
    b = workloads.weights(m, seed=seed + 11) if weighted else workloads.weights(m)
    a, b = a.astype(np.float64), b.astype(np.float64)
    return a / a.sum(), X, b / b.sum(), Y


def test_cost_matrix_direct_differences():
    X = np.array([[0.0, 0.0], [1.0, 2.0]])
    Y = np.array([[3.0, 4.0], [-1.0, 0.5], [1.0, 2.0]])
    C = cost_matrix(X, Y)
    exp = np.array([[25.0, 1.25, 5.0], [8.0, 6.25, 0.0]])
    np.testing.assert_allclose(C, exp, rtol=0, atol=1e-15)


def test_marginals_at_exit():
    """Alg. 1 returns once |P1 - a|_1 <= tau; the g-update makes P^T 1 = b to
    rounding (exact invariant of the alternating updates)."""
    a, X, b, Y = _small()
    C = cost_matrix(X, Y)
    eps = 0.1 * C.mean()
    res = oracle.sinkhorn(a, X, b, Y, eps, tau=1e-9)
    assert res.converged and res.err <= 1e-9
    row, col = oracle.marginal_errors(res.f, res.g, C, eps, a, b)
    assert row <= 1e-9
    assert col <= 1e-13
    assert abs(row - res.err) <= 1e-14


def test_loop_condition_is_err_above_tau():
    """The loop runs while err > tau: a loose tau stops earlier and its
    returned iterate already satisfies err <= tau, the previous one does not."""
    a, X, b, Y = _small(seed=3)
    C = cost_matrix(X, Y)
    eps = 0.05 * C.mean()
    r = oracle.sinkhorn(a, X, b, Y, eps, tau=1e-3)
    assert r.iters >= 2 and r.err <= 1e-3
    prev = oracle.sinkhorn(a, X, b, Y, eps, tau=0.0, n_iter=r.iters - 1)
    assert prev.err > 1e-3


def test_matches_textbook_scaling_iterations():
    """Log-domain Sinkhorn equals the textbook Sinkhorn-Knopp matrix scaling
    u = a / (K v), v = b / (K^T u) with K = exp(-C/eps), through f = eps log u,
    g = eps log v, iterate by iterate (moderate eps, no underflow)."""
    a, X, b, Y = _small(seed=1)
    C = cost_matrix(X, Y)
    eps = 0.5 * C.mean()
    Kmat = np.exp(-C / eps)
    v = np.ones(C.shape[1])
    for it in (1, 2, 3, 7):
        vv = v.copy()
        for _ in range(it):
            u = a / (Kmat @ vv)
            vv = b / (Kmat.T @ u)
        res = oracle.sinkhorn(a, X, b, Y, eps, tau=0.0, n_iter=it)
        np.testing.assert_allclose(res.f, eps * np.log(u), rtol=0, atol=1e-11)
        np.testing.assert_allclose(res.g, eps * np.log(vv), rtol=0, atol=1e-11)


def test_warm_start_is_g_only():
    """f_init cannot change the iterates (the first f-update overwrites f);
    g_init does."""
    a, X, b, Y = _small(seed=2)
    C = cost_matrix(X, Y)
    eps = 0.2 * C.mean()
    r0 = oracle.sinkhorn(a, X, b, Y, eps, 0.0, n_iter=3)
    r1 = oracle.sinkhorn(a, X, b, Y, eps, 0.0, f_init=np.full(60, 5.0), n_iter=3)
    np.testing.assert_array_equal(r0.f, r1.f)
    r2 = oracle.sinkhorn(a, X, b, Y, eps, 0.0, g_init=np.linspace(-1, 1, 50), n_iter=1)
    assert np.abs(r2.f - oracle.sinkhorn(a, X, b, Y, eps, 0.0, n_iter=1).f).max() > 1e-6


def _brute_force(C):
    n = C.shape[0]
    best, perm = math.inf, None
    for p in itertools.permutations(range(n)):
        v = C[np.arange(n), p].sum()
        if v < best:
            best, perm = v, np.array(p)
    return best / n, perm


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_eps_brute_force(seed):
    """As eps -> 0 the entropic plan concentrates on the optimal assignment:
    row argmax of P is the optimal permutation (found by enumerating all 7!
    permutations), and OT <= <P, C> <= OT + eps log m (compare the entropic
    objective at P_eps and at the optimal permutation, H(P) <= log nm); the
    row-marginal slack tau adds at most 2 tau max C to either side."""
    n = 7
    rng = np.random.default_rng(100 + seed)
    X = rng.uniform(-1, 1, (n, 2)).astype(np.float32)
    perm = rng.permutation(n)
    Y = (X[perm] + 0.05 * rng.standard_normal((n, 2))).astype(np.float32)
    a = np.full(n, 1.0 / n)
    C = cost_matrix(X, Y)
    ot, sigma = _brute_force(C)
    eps = 0.05 * C.mean()
    tau = 1e-6
    res = oracle.sinkhorn(a, X, a, Y, eps, tau=tau, max_iter=50_000)
    assert res.converged
    P = oracle.coupling(res.f, res.g, C, eps)
    np.testing.assert_array_equal(P.argmax(axis=1), sigma)
    pc = float((P * C).sum())
    slack = 2 * tau * C.max()
    assert ot - slack <= pc <= ot + eps * math.log(n) + slack


def test_large_eps_expansion():
    """For large eps, eps (P_ij/(a_i b_j) - 1) -> 2 (x_i - xbar)^T (y_j - ybar)
    with error O(1/eps), and T(x_i) -> ybar + (2/eps) Cov_b(Y) (x_i - xbar)
    with error O(1/eps^2) (first-order expansion of the Gibbs kernel; the
    double-centred cost is -2 <x - xbar, y - ybar>)."""
    a, X, b, Y = _small(seed=4, n=40, m=30, d=3)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    xbar, ybar = a @ Xd, b @ Yd
    lin = 2.0 * (Xd - xbar) @ (Yd - ybar).T
    covY = ((Yd - ybar) * b[:, None]).T @ (Yd - ybar)
    C = cost_matrix(X, Y)
    errs_p, errs_t = [], []
    for eps in (50.0 * C.mean(), 500.0 * C.mean()):
        res = oracle.sinkhorn(a, X, b, Y, eps, tau=1e-13, max_iter=1000)
        P = oracle.coupling(res.f, res.g, C, eps)
        errs_p.append(np.abs(eps * (P / np.outer(a, b) - 1.0) - lin).max())
        T = oracle.entropic_map(X, Y, res.g, eps)
        Tlin = ybar + (2.0 / eps) * (Xd - xbar) @ covY.T
        errs_t.append(np.abs(T - Tlin).max())
    assert 6.0 < errs_p[0] / errs_p[1] < 15.0
    assert 60.0 < errs_t[0] / errs_t[1] < 150.0
    assert errs_p[1] < 0.01 * np.abs(lin).max()


def _quantile_cloud(n, var, shift=0.0):
    return (shift + math.sqrt(var) * norm.ppf((np.arange(n) + 0.5) / n))[:, None]


@pytest.mark.parametrize("eps", [0.5, 2.0])
def test_gaussian_closed_form_1d(eps):
    """Entropic OT between N(m1, A) and N(m2, B) under cost |x - y|^2 is a
    Gaussian plan whose precision has off-diagonal -2/eps, giving the
    cross-covariance c = (-eps + sqrt(eps^2 + 16 A B))/4 and the linear
    entropic map T(x) = m2 + (c/A)(x - m1).  Quantile points make the
    empirical measures close to the Gaussians."""
    A, B, m1, m2 = 1.0, 2.25, 0.3, -0.7
    n = 3000
    X = _quantile_cloud(n, A, m1).astype(np.float32)
    Y = _quantile_cloud(n, B, m2).astype(np.float32)
    a = np.full(n, 1.0 / n)
    res = oracle.sinkhorn(a, X, a, Y, eps, tau=1e-10)
    T = oracle.entropic_map(X, Y, res.g, eps)[:, 0]
    x = X[:, 0].astype(np.float64)
    c = (-eps + math.sqrt(eps * eps + 16.0 * A * B)) / 4.0
    slope = np.polyfit(x - x.mean(), T, 1)[0]
    assert abs(slope - c / A) / (c / A) < 3e-3
    core = np.abs(x - m1) < 1.5
    pred = m2 + (c / A) * (x - m1)
    assert np.abs(T - pred)[core].max() < 1e-2


def test_gaussian_closed_form_2d():
    """d = 2: T(x) = m2 + C_eps^T A^{-1} (x - m1) with C_eps = 1/2 A^{1/2} D
    A^{-1/2} - (eps/4) I, D = (4 A^{1/2} B A^{1/2} + eps^2/4 I)^{1/2}
    (Janati et al. 2020, balanced case, rescaled to cost |.|^2).  Statistical
    check on random samples."""
    rng = np.random.default_rng(5)
    A = np.array([[1.0, 0.3], [0.3, 0.6]])
    B = np.array([[2.0, -0.4], [-0.4, 1.0]])
    n, eps = 2500, 1.0

    def sqrtm(M):
        w, V = np.linalg.eigh(M)
        return (V * np.sqrt(w)) @ V.T

    X = (rng.standard_normal((n, 2)) @ np.linalg.cholesky(A).T).astype(np.float32)
    Y = (rng.standard_normal((n, 2)) @ np.linalg.cholesky(B).T).astype(np.float32)
    a = np.full(n, 1.0 / n)
    res = oracle.sinkhorn(a, X, a, Y, eps, tau=1e-8)
    T = oracle.entropic_map(X, Y, res.g, eps)
    Ah = sqrtm(A)
    D = sqrtm(4.0 * Ah @ B @ Ah + (eps * eps / 4.0) * np.eye(2))
    Ce = 0.5 * Ah @ D @ np.linalg.inv(Ah) - (eps / 4.0) * np.eye(2)
    M = Ce.T @ np.linalg.inv(A)
    Xc = X.astype(np.float64) - X.mean(0)
    Mfit = np.linalg.lstsq(Xc, T - T.mean(0), rcond=None)[0].T
    assert np.abs(Mfit - M).max() / np.abs(M).max() < 6e-2


def test_translation_invariance():
    """Shifting Y by v leaves P unchanged (the cost changes by a row term plus
    a column term, absorbed by the potentials) and shifts the map by v;
    shifting both clouds leaves f and g unchanged."""
    a, X, b, Y = _small(seed=6)
    eps = 0.1 * cost_matrix(X, Y).mean()
    v = np.array([0.75, -1.5, 0.25])
    r0 = oracle.sinkhorn(a, X, b, Y, eps, 0.0, n_iter=400)
    Y1 = Y.astype(np.float64) + v
    r1 = oracle.sinkhorn(a, X, b, Y1, eps, 0.0, n_iter=400)
    P0 = oracle.coupling(r0.f, r0.g, cost_matrix(X, Y), eps)
    P1 = oracle.coupling(r1.f, r1.g, cost_matrix(X, Y1), eps)
    np.testing.assert_allclose(P1, P0, rtol=1e-8, atol=1e-14)
    T0 = oracle.entropic_map(X, Y, r0.g, eps)
    T1 = oracle.entropic_map(X, Y1, r1.g, eps)
    np.testing.assert_allclose(T1, T0 + v, rtol=0, atol=1e-10)
    r2 = oracle.sinkhorn(a, X.astype(np.float64) + v, b, Y1, eps, 0.0, n_iter=400)
    np.testing.assert_allclose(r2.f, r0.f, rtol=0, atol=1e-9)
    np.testing.assert_allclose(r2.g, r0.g, rtol=0, atol=1e-9)


def test_map_jacobian_is_scaled_covariance():
    """The Jacobian of the entropic map is eps'^{-1} Cov(Y | X = x) for the
    1/2-cost (Lemma on Lipschitz bounds, App. A); with h = |.|^2 the
    exponent carries 2/eps, so DT(x) = (2/eps) Cov_{p(x)}(Y), symmetric PSD.
    Checked by central finite differences at out-of-sample points."""
    a, X, b, Y = _small(seed=7)
    eps = 0.3 * cost_matrix(X, Y).mean()
    res = oracle.sinkhorn(a, X, b, Y, eps, tau=1e-10)
    Yd = Y.astype(np.float64)
    for x in (np.array([0.2, -0.1, 0.4]), np.array([-1.0, 0.5, 0.0])):
        h = 1e-5
        J = np.zeros((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (oracle.entropic_map((x + e)[None], Y, res.g, eps)[0]
                       - oracle.entropic_map((x - e)[None], Y, res.g, eps)[0]) / (2 * h)
        p = oracle.map_weights(x[None], Y, res.g, eps)[0]
        mu = p @ Yd
        cov = ((Yd - mu) * p[:, None]).T @ (Yd - mu)
        np.testing.assert_allclose(J, (2.0 / eps) * cov, rtol=1e-6, atol=1e-8)
        assert np.abs(J - J.T).max() < 1e-7


def test_duality_gap_closes():
    """At the fixed point, the primal <P, C> + eps sum P (log P - 1) equals the
    dual <f, a> + <g, b> - eps sum P (eq. entdual)."""
    a, X, b, Y = _small(seed=8)
    C = cost_matrix(X, Y)
    eps = 0.1 * C.mean()
    res = oracle.sinkhorn(a, X, b, Y, eps, tau=1e-12)
    P = oracle.coupling(res.f, res.g, C, eps)
    gap = oracle.primal_objective(P, C, eps) - oracle.dual_objective(res.f, res.g, C, eps, a, b)
    assert abs(gap) < 1e-10 * max(1.0, abs(oracle.dual_objective(res.f, res.g, C, eps, a, b)))


def test_spd_identity_coupling():
    """Y = X G^T with G symmetric positive definite: the optimal matching is the
    identity (Prop. on the blurred-image benchmark, Sec. 5.3, via Brenier), so
    Tr(n P) -> 1 as eps -> 0, increasing as eps decreases."""
    X, Y = workloads.spd_pair(seed=9, n=128, d=6)
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    C = cost_matrix(X, Y)
    traces = []
    for beta in (1.0, 0.3, 0.1):
        eps = beta * C.mean() / 20.0
        res = oracle.sinkhorn(a, X, a, Y, eps, tau=1e-4, max_iter=100_000)
        P = oracle.coupling(res.f, res.g, C, eps)
        traces.append(float(np.trace(P)))
    assert traces[0] < traces[1] < traces[2]
    assert traces[2] > 0.99
