"""Parity at the benchmark's full size (n = m = 16384, d = 64, FP32, the same
launch configuration bench.py times), on sampled outputs that the FP64
oracle computes one by one: a row of the f-update needs all m columns and a
column of the g-update all n rows, which the oracle evaluates exactly for a
seeded sample."""
import numpy as np
import pytest

import oracle
from oracle.sinkhorn import cost_matrix, softmin_rows
import workloads
from tests.parity import map_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 16384
D = 64


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    X, Y = workloads.gmm(seed=2, n=N, m=N, d=D)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
    return P, X, Y, cl


def _moments_mean_cost(X, Y):
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    return (Xd ** 2).sum(1).mean() + (Yd ** 2).sum(1).mean() - 2 * Xd.mean(0) @ Yd.mean(0)


def test_mean_cost_full(setup):
    P, X, Y, cl = setup
    assert abs(cl.mean_cost / _moments_mean_cost(X, Y) - 1) < 1e-9


def test_half_steps_sampled(setup):
    """f' = f-update(g) at 256 sampled rows and g' = g-update(f') at 256
    sampled columns, each against the FP64 soft-min over the full other side."""
    P, X, Y, cl = setup
    eps = cl.mean_cost / 20.0
    f, g, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=4)
    f2, g2, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=1, g_init=g)
    g64 = g.cpu().numpy().astype(np.float64)
    f2_64 = f2.cpu().numpy().astype(np.float64)
    g2_64 = g2.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(12)
    rows = rng.choice(N, 256, replace=False)
    cols = rng.choice(N, 256, replace=False)
    la = np.log(1.0 / N)
    ref_f = eps * la - eps * softmin_rows(cost_matrix(X[rows], Y), g64, eps)
    ref_g = eps * la - eps * softmin_rows(cost_matrix(Y[cols], X), f2_64, eps)
    scale_f = max(np.abs(f2_64).max(), eps)
    scale_g = max(np.abs(g2_64).max(), eps)
    ef = np.abs(f2_64[rows] - ref_f).max() / scale_f
    eg = np.abs(g2_64[cols] - ref_g).max() / scale_g
    print(f"full-size half-steps: f err {ef:.2e}, g err {eg:.2e}", flush=True)
    assert ef < 1e-4 and eg < 1e-4


def test_progot_full_sampled(setup):
    """The benchmark's solve: K = 8, tau = 1e-3.  Final FP64 marginals meet
    tau; the final map at 256 sampled points matches the FP64 entropic map of
    the GPU-fitted (X^(K-1), g^(K-1), eps_{K-1})."""
    P, X, Y, cl = setup
    f, G, TX, info = P.progot_solve(cl, 8, tau_first=1e-3, tau_last=1e-3)
    print(f"full-size ProgOT: iters {info.iters}, eps {info.eps}", flush=True)
    assert info.converged
    row, col, _ = P.marginal_check(cl, f, G[-1], info.eps[-1])
    assert row <= 1e-3 * 1.01 and col <= 1e-4
    Xlast = cl.xk().cpu().numpy()
    rows = np.random.default_rng(13).choice(N, 256, replace=False)
    ref = oracle.entropic_map(Xlast[rows], Y, G[-1].cpu().numpy().astype(np.float64),
                              float(info.eps[-1]), alpha=1.0)
    assert map_err(TX.cpu().numpy()[rows], ref, Y) < 1e-3


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_spd_identity_trace_at_scale(setup, prec):
    """Y = X G^T with G SPD (eigenvalues in [1, 4]): the optimal matching is
    the identity (Prop. on the blurred-image benchmark, via Brenier), so the
    trace of the final ProgOT coupling between X^(K-1) and Y rises to 1 as
    theta shrinks.  A property that holds at any size, checked at n = 65536
    (d = 16) in O(n d) from the GPU's potentials: Tr P = sum_i
    exp((f_i + g_i - |x_i - y_i|^2)/eps).  Measured on MI355X: 0.232, 0.991,
    1.000 at theta = 1, 0.3, 0.1 (both forms)."""
    P = setup[0]
    X, Y = workloads.spd_pair(seed=21, n=65536, d=16, cond=4.0)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    traces = []
    for theta in (1.0, 0.3, 0.1):
        f, G, _, info = P.progot_solve(cl, 4, theta=theta, tau_first=1e-3, tau_last=1e-3,
                                       want_TX=False)
        assert info.converged
        Xl = cl.xk().cpu().numpy().astype(np.float64)
        cii = ((Xl - Y.astype(np.float64)) ** 2).sum(1)
        f64 = f.cpu().numpy().astype(np.float64)
        g64 = G[-1].cpu().numpy().astype(np.float64)
        traces.append(float(np.exp((f64 + g64 - cii) / float(info.eps[-1])).sum()))
    print(f"SPD identity {prec}: traces {traces}", flush=True)
    assert traces[0] < traces[1] < traces[2]
    assert traces[2] > 0.999
