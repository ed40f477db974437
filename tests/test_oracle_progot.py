"""Pins of the FP64 ProgOT oracle, its progressive map and its schedules."""
import math
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest
from scipy.stats import norm

import oracle
from oracle import schedules
from oracle.sinkhorn import cost_matrix
import workloads

GOLDEN = Path(__file__).parent / "golden"


def _golden_alpha():
    rows = {}
    for line in (GOLDEN / "alpha_schedules_K4.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        kind, rest = line.split(None, 1)
        al, tt = rest.split("|")
        rows[kind] = ([float(Fraction(x)) for x in al.split()], [float(Fraction(x)) for x in tt.split()])
    return rows


@pytest.mark.parametrize("kind", ["constant", "accelerated"])
def test_alpha_schedule_golden(kind):
    alpha, t = _golden_alpha()[kind]
    np.testing.assert_allclose(schedules.alpha_schedule(4, kind), alpha, rtol=0, atol=1e-15)
    np.testing.assert_allclose(schedules.progress(schedules.alpha_schedule(4, kind)), t,
                               rtol=0, atol=1e-15)


@pytest.mark.parametrize("K", [1, 2, 3, 8, 16])
def test_alpha_schedule_closed_forms(K):
    """Constant speed: t_k = (k+1)/K, equal increments; accelerated: t_k =
    ((k+1)/K)^2, increasing increments; decelerated: alpha = 1/e until the
    complete last step, decreasing increments (Sec. 4 definitions)."""
    ks = np.arange(1, K + 1)
    np.testing.assert_allclose(schedules.progress(schedules.alpha_schedule(K, "constant")),
                               ks / K, atol=1e-14)
    np.testing.assert_allclose(schedules.progress(schedules.alpha_schedule(K, "accelerated")),
                               (ks / K) ** 2, atol=1e-14)
    dec = schedules.alpha_schedule(K, "decelerated")
    assert dec[-1] == 1.0 and np.all(dec[:-1] == 1.0 / math.e)
    tdec = schedules.progress(dec)
    if K >= 3:
        inc = np.diff(np.concatenate([[0.0], tdec[:-1]]))
        assert np.all(np.diff(inc) < 0)


def test_eps_mean_cost_closed_form():
    """mean_ij |x_i - y_j|^2 = mean |x|^2 + mean |y|^2 - 2 xbar . ybar."""
    X, Y = workloads.gmm(seed=11, n=300, m=200, d=5)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    closed = (Xd ** 2).sum(1).mean() + (Yd ** 2).sum(1).mean() - 2 * Xd.mean(0) @ Yd.mean(0)
    assert abs(schedules.eps_mean_cost(X, Y, theta=0.5) - 0.5 * closed / 20) < 1e-12 * closed


def test_tau_schedule():
    np.testing.assert_allclose(schedules.tau_schedule(4, 1e-2, 1e-3), [1e-2, 7e-3, 4e-3, 1e-3])
    assert schedules.tau_schedule(1, 1e-2, 1e-3)[0] == 1e-3


def test_c1_holdout_same_mixture():
    """The hold-out targets are fresh draws of the same target mixture: a
    large hold-out sample matches the mixture's mean (equal component
    weights) and the training targets' statistics."""
    import math
    rng = np.random.default_rng(1)
    rng.standard_normal((1024, 4))
    mu = rng.standard_normal((4, 4)) * 2.0
    Yt = workloads.c1_holdout(seed=1, m_test=200_000, test_seed=101).astype(np.float64)
    assert np.abs(Yt.mean(0) - mu.mean(0)).max() < 0.03
    Y = workloads.c1(seed=1)[1].astype(np.float64)
    sd = Yt.std(0)
    assert (np.abs(Y.mean(0) - Yt.mean(0)) < 4 * sd / math.sqrt(Y.shape[0]) + 0.15 * sd).all()
    # a different test seed gives different points
    assert not np.allclose(workloads.c1_holdout(seed=1, m_test=10, test_seed=5),
                           workloads.c1_holdout(seed=1, m_test=10, test_seed=6))


def test_eps_scheduler_structure():
    """Alg. 4 on a small C1-type problem: sigma is the intra-target mean cost
    / 20 (= 2 (mean |y|^2 - |ybar|^2)/20); the schedule starts at beta0 eps0,
    ends at s_{p*} sigma and, for constant speed, is linear in k/(K-1)."""
    X, Y = workloads.c1(seed=1, n=200, m=200)
    Yt = workloads.c1_holdout(seed=1, n=200, m_test=200, test_seed=101)
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    alpha = schedules.alpha_schedule(4, "constant")
    sched, info = schedules.eps_scheduler(a, X, a, Y, alpha, Yt, beta0=5.0)
    Yd = Y.astype(np.float64)
    sigma = 2 * ((Yd ** 2).sum(1).mean() - (Yd.mean(0) ** 2).sum()) / 20
    assert abs(info["sigma"] - sigma) < 1e-10 * sigma
    assert info["p_star"] == int(np.argmin(info["errors"]))
    s_star = 2.0 ** (info["p_star"] - 3)
    assert abs(sched[0] - 5.0 * info["eps0"]) < 1e-12 * sched[0]
    assert abs(sched[-1] - s_star * sigma) < 1e-12 * sched[-1]
    lin = 5.0 * info["eps0"] + (s_star * sigma - 5.0 * info["eps0"]) * np.arange(4) / 3
    np.testing.assert_allclose(sched, lin, rtol=1e-12)


def test_eps_scheduler_eps0_closed_form():
    """Alg. 4's eps_0 is the source-target mean cost / 20; the mean cost has
    the moments closed form mean |x|^2 + mean |y|^2 - 2 xbar . ybar, formed
    here from the clouds (not read from the scheduler), and the first step of
    a constant-speed schedule is beta0 eps_0."""
    X, Y = workloads.c1(seed=1, n=180, m=150)
    Yt = workloads.c1_holdout(seed=1, n=180, m_test=120, test_seed=101)
    a = np.full(X.shape[0], 1.0 / X.shape[0])
    b = np.full(Y.shape[0], 1.0 / Y.shape[0])
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    cbar = (Xd ** 2).sum(1).mean() + (Yd ** 2).sum(1).mean() - 2 * Xd.mean(0) @ Yd.mean(0)
    for beta0 in (5.0, 2.0):
        sched, info = schedules.eps_scheduler(a, X, b, Y, schedules.alpha_schedule(4), Yt,
                                              beta0=beta0)
        assert abs(sched[0] - beta0 * cbar / 20) < 1e-12 * sched[0]
        assert abs(info["eps0"] - cbar / 20) < 1e-12 * cbar


def _weighted_target(seed=1, m=160, m_test=150):
    X, Y = workloads.c1(seed=seed, n=200, m=m)
    Yt = workloads.c1_holdout(seed=seed, n=200, m_test=m_test, test_seed=101)
    rng = np.random.default_rng(7)
    b = rng.uniform(0.5, 1.5, m)
    return X, Y, b / b.sum(), Yt


def test_eps_scheduler_score_large_eps_limit():
    """The hold-out score sum |y~ - T(y~)|^2 at grid scale eps = s sigma.  As
    eps grows the Y -> Y potentials carry the weights b and the map tends to
    T(y~) = ybar_b + (2/eps) Cov_b(Y)(y~ - ybar_b) + O(1/eps^2) (the
    large-eps expansion pinned for Sinkhorn itself), so the score tends to
    sum |y~ - ybar_b|^2 with the first-order gap
    -(4/eps) sum (y~ - ybar_b)^T Cov_b(Y) (y~ - ybar_b); the relative error
    of that gap shrinks ~10x per decade of eps."""
    X, Y, b, Yt = _weighted_target()
    a = np.full(X.shape[0], 1.0 / X.shape[0])
    Yd = Y.astype(np.float64)
    ybar = b @ Yd
    Z = Yd - ybar
    cov = (Z * b[:, None]).T @ Z
    D = Yt.astype(np.float64) - ybar
    limit = (D ** 2).sum()
    quad = np.einsum("ij,jk,ik->", D, cov, D)
    grid = [1e3, 1e4]
    _, info = schedules.eps_scheduler(a, X, b, Y, schedules.alpha_schedule(4), Yt,
                                      s_grid=grid, tau=1e-10)
    rel = []
    for s, score in zip(grid, info["errors"]):
        first_order = -4.0 / (s * info["sigma"]) * quad
        assert abs(score - limit) < 0.02 * limit
        rel.append(abs((score - limit) / first_order - 1.0))
    assert rel[0] < 5e-3 and rel[1] < 5e-4
    assert 5.0 < rel[0] / rel[1] < 20.0


def _problem(seed=21, n=150, m=120, d=3):
    X, Y = workloads.gmm(seed=seed, n=n, m=m, d=d, n_comp=3)
    a = np.full(n, 1.0 / n)
    b = np.full(m, 1.0 / m)
    return a, X, b, Y


def test_k1_is_sinkhorn_plus_map():
    """K = 1 (alpha_0 = 1): ProgOT is one Sinkhorn solve followed by the
    entropic map (Def. of ProgOT)."""
    a, X, b, Y = _problem()
    r = oracle.progot(a, X, b, Y, K=1, tau=1e-6)
    eps = schedules.eps_mean_cost(X, Y)
    s = oracle.sinkhorn(a, X, b, Y, eps, 1e-6)
    np.testing.assert_allclose(r.f, s.f, atol=1e-12)
    np.testing.assert_allclose(r.G[0], s.g, atol=1e-12)
    np.testing.assert_allclose(r.TX, oracle.entropic_map(X, Y, s.g, eps), atol=1e-12)
    assert r.alpha[0] == 1.0 and r.iters == [s.iters]


def test_progressive_map_reproduces_training_trajectory():
    """Alg. 3 evaluated at the training points reproduces the end of Alg. 2's
    trajectory X^(K) (both apply S_k = (1 - alpha_k) Id + alpha_k T_k in
    turn, the last alpha being 1)."""
    a, X, b, Y = _problem(seed=22)
    r = oracle.progot(a, X, b, Y, K=4, tau=1e-4)
    Tx = oracle.progot_map(X, Y, r.G, r.eps, r.alpha)
    np.testing.assert_allclose(Tx, r.TX, atol=1e-10)


def test_progot_step_marginals_and_eps():
    """Every solve ends with err <= tau_k; eps_k is the per-step mean-cost rule
    on the moved cloud; the final coupling's marginals meet tau."""
    a, X, b, Y = _problem(seed=23)
    taus = schedules.tau_schedule(4, 1e-2, 1e-4)
    r = oracle.progot(a, X, b, Y, K=4, tau=taus)
    assert all(e <= t for e, t in zip(r.errs, taus))
    assert r.final_row_err <= 1e-4 and r.final_col_err < 1e-12
    np.testing.assert_allclose(r.eps[0], schedules.eps_mean_cost(X, Y), rtol=1e-12)
    np.testing.assert_allclose(r.eps[-1], schedules.eps_mean_cost(r.X_last, Y), rtol=1e-12)
    assert r.eps[-1] < r.eps[0]


def test_last_step_starts_cold():
    """Alg. 2 warm-starts solve k from (1 - alpha_k) times the previous
    potentials; the last step has alpha = 1, so in fixed-iteration mode the
    last solve is exactly a cold Sinkhorn run (zero initial potentials) on
    the moved cloud X^(K-1), whatever the earlier steps left behind."""
    a, X, b, Y = _problem(seed=25)
    for K in (2, 3):
        r = oracle.progot(a, X, b, Y, K=K, n_iter=6)
        s = oracle.sinkhorn(a, r.X_last, b, Y, r.eps[-1], 0.0, n_iter=6)
        np.testing.assert_allclose(r.G[-1], s.g, rtol=0, atol=1e-12 * np.abs(s.g).max())
        np.testing.assert_allclose(r.f, s.f, rtol=0, atol=1e-12 * np.abs(s.f).max())


def test_warm_start_variants_agree():
    """Warm starting changes iteration counts, not solutions (to within the
    tolerance)."""
    a, X, b, Y = _problem(seed=24)
    r1 = oracle.progot(a, X, b, Y, K=3, tau=1e-7)
    r2 = oracle.progot(a, X, b, Y, K=3, tau=1e-7, warm_start="alpha_prev")
    scale = np.abs(r1.TX).max()
    assert np.abs(r1.TX - r2.TX).max() < 1e-4 * scale


def test_progot_recovers_monotone_map_1d():
    """1-D: the OT map between quantile clouds of N(0, 1) and N(1, 4) is the
    monotone rearrangement x -> 1 + 2x.  With a small per-step eps, ProgOT's
    final points approach it."""
    n = 400
    q = norm.ppf((np.arange(n) + 0.5) / n)
    X = q[:, None].astype(np.float32)
    Y = (1.0 + 2.0 * q)[:, None].astype(np.float32)
    a = np.full(n, 1.0 / n)
    r = oracle.progot(a, X, a, Y, K=4, theta=0.2, tau=1e-4)
    target = 1.0 + 2.0 * X[:, 0].astype(np.float64)
    core = np.abs(q) < 1.5
    err_prog = np.abs(r.TX[core, 0] - target[core]).max()
    assert err_prog < 0.03
    # a single entropic map at the first step's eps is more biased (Sec. 3)
    s = oracle.sinkhorn(a, X, a, Y, r.eps[0], 1e-4)
    T1 = oracle.entropic_map(X, Y, s.g, r.eps[0])
    assert err_prog < np.abs(T1[core, 0] - target[core]).max()


def test_progot_spd_identity_trace():
    """Y = X G^T, G SPD: the ProgOT coupling also recovers the identity
    matching as theta shrinks (Prop. on the blurred-image benchmark)."""
    X, Y = workloads.spd_pair(seed=12, n=96, d=5)
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    r = oracle.progot(a, X, a, Y, K=4, theta=0.1, tau=1e-5)
    P = oracle.coupling(r.f, r.G[-1], cost_matrix(r.X_last, Y), r.eps[-1])
    assert np.trace(P) > 0.99
