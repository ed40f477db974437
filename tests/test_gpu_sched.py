"""Alg. 4 (the eps-scheduler) on the GPU against the FP64 oracle's Alg. 4.

On the small ProgOT workload (n = m = 1024, d = 4, K = 4, hold-out targets:
1024 fresh draws of the target mixture): eps_0 and sigma agree to rounding,
the grid scores to the FP32 map's accuracy, the selected scale is the same,
and so the schedule agrees; ProgOT run with the GPU schedule matches the
oracle run with the oracle's schedule."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import map_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    return P


@pytest.mark.parametrize("K,alpha_sched", [(4, "constant"), (5, "accelerated"), (1, "constant")])
def test_eps_schedule_matches_oracle(P, K, alpha_sched):
    X, Y = workloads.c1(seed=1)
    Yt = workloads.c1_holdout(seed=1, test_seed=101)
    n, m = X.shape[0], Y.shape[0]
    a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
    tau = 1e-3
    alpha = oracle.schedules.alpha_schedule(K, alpha_sched)
    ref, info = oracle.schedules.eps_scheduler(a, X, b, Y, alpha, Yt, beta0=5.0, tau=tau)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
    out = P.eps_schedule(cl, P.to_device(Yt), K, alpha_sched=alpha_sched, beta0=5.0, tau=tau)
    print(f"case K={K} {alpha_sched}: p* gpu {out.p_star} oracle {info['p_star']}; "
          f"scores gpu {np.array(out.errors)} oracle {np.array(info['errors'])}", flush=True)
    assert out.status == 0
    # the scores are sums over 1024 hold-out points of FP32 maps (~1e-6
    # relative each) at tau-stopped potentials that may stop one iteration
    # apart: 1e-3 relative
    np.testing.assert_allclose(out.errors, info["errors"], rtol=1e-3)
    srt = np.sort(info["errors"])
    if srt[1] > srt[0] * (1 + 1e-2):      # a clear winner: the same scale
        assert out.p_star == info["p_star"]
        # eps_0 and sigma agree to FP64 rounding; t_k comes from the
        # library's FP32 alpha schedule (1/3 in FP32 is 1e-8 off)
        np.testing.assert_allclose(out.eps, ref, rtol=1e-7)
    else:                                  # near-tie: either choice is valid
        assert abs(info["errors"][out.p_star] - srt[0]) <= 1e-2 * srt[0]


def test_progot_with_gpu_schedule(P):
    """ProgOT fed the GPU schedule equals the oracle's ProgOT fed the
    oracle's schedule (same selected scale, so the same eps_k)."""
    X, Y = workloads.c1(seed=1)
    Yt = workloads.c1_holdout(seed=1, test_seed=101)
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    K, tau = 4, 1e-3
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
    sched = P.eps_schedule(cl, P.to_device(Yt), K, tau=tau)
    eps32 = np.asarray(sched.eps, dtype=np.float32).astype(np.float64)
    f, G, TX, info = P.progot_solve(cl, K, eps=eps32, tau_first=tau, tau_last=tau)
    ref = oracle.progot(a, X, a, Y, K, eps=eps32, tau=tau)
    assert info.converged
    np.testing.assert_allclose(info.eps, ref.eps, rtol=1e-6)
    assert map_err(TX.cpu().numpy(), ref.TX, Y) < 1e-3


def test_eps_schedule_weighted_and_nonconverged(P):
    """Weighted targets reach the grid solves (b on both sides), and a grid
    solve stopped by max_iter is reported as a warning with valid output."""
    X, Y = workloads.gmm(seed=31, n=400, m=300, d=8)
    b = workloads.weights(300, seed=32)
    Yt = workloads.gmm(seed=31, n=400, m=300, d=8)[1][:200]
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), b=P.to_device(b))
    out = P.eps_schedule(cl, P.to_device(Yt), 3, tau=1e-3)
    bb = b.astype(np.float64)
    bb /= bb.sum()
    ref, info = oracle.schedules.eps_scheduler(np.full(400, 1 / 400), X, bb, Y,
                                               oracle.schedules.alpha_schedule(3), Yt, beta0=5.0,
                                               tau=1e-3)
    np.testing.assert_allclose(out.errors, info["errors"], rtol=1e-3)
    few = P.eps_schedule(cl, P.to_device(Yt), 3, tau=1e-9, max_iter=3)
    assert few.status == 1
    assert all(np.isfinite(few.eps))


@pytest.mark.parametrize("tau,max_iter", [(1e-3, 10_000), (1e-9, 1), (1e-9, 3), (1e-9, 5),
                                          (1e-6, 40)])
def test_grid_solves_match_single_problem(P, tau, max_iter):
    """Each grid solve of the scheduler (grid points advanced together, the
    stop rule evaluated on the device, several iterations per read-back)
    stops at the same iterate as the single-problem Sinkhorn solve with that
    scale's eps, so its hold-out score equals the score of that solve's map
    up to the order of one FP64 sum.  max_iter 1, 3, 5 cover the last-iterate
    probe inside and right after the first block of iterations."""
    X, Y = workloads.gmm(seed=31, n=400, m=300, d=8)
    b = workloads.weights(300, seed=32)
    Yt = workloads.gmm(seed=33, n=400, m=300, d=8)[1][:200]
    Yd, bd, Ytd = P.to_device(Y), P.to_device(b), P.to_device(Yt)
    cl = P.prepare_clouds(P.to_device(X), Yd, b=bd)
    grid = [2.0 ** k for k in range(-3, 4)]
    out = P.eps_schedule(cl, Ytd, 3, s_grid=grid, tau=tau, max_iter=max_iter)
    cy = P.prepare_clouds(Yd, Yd, a=bd, b=bd)
    sigma = cy.mean_cost / 20.0
    ref, conv = [], []
    for s in grid:
        eps = float(np.float32(s * sigma))
        _, g, info = P.sinkhorn_solve(cy, eps, tau=tau, max_iter=max_iter)
        ty = P.entropic_map(cy, g, eps, Ytd).cpu().numpy().astype(np.float64)
        ref.append(((Yt.astype(np.float32).astype(np.float64) - ty) ** 2).sum())
        conv.append(info.converged)
    print(f"case tau={tau} max_iter={max_iter}: scores {np.array(out.errors)} ref {np.array(ref)}",
          flush=True)
    np.testing.assert_allclose(out.errors, ref, rtol=1e-12)
    assert out.status == (0 if all(conv) else 1)
