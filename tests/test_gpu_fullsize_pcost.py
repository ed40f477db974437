"""Parity of the general-cost path at the benchmark's size for it
(`bench.py --workload pcost_4i_d47`: n = 11000, m = 2800, d = 47,
h = (1/p)|.|_p^p with p = 1.5, K = 4, theta = 2^-4, tau = 1e-3), in the same
launch configuration, on outputs the FP64 oracle computes one by one: the
f-update at sampled rows needs all m columns of C, the g-update at sampled
columns all n rows, and the map at a sampled point all m targets."""
import numpy as np
import pytest

import oracle
from oracle import pcost
from oracle.sinkhorn import softmin_rows
import workloads
from tests.parity import map_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, M, D, PEXP = 11000, 2800, 47, 1.5


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    X, Y = workloads.gmm(seed=12, n=N, m=M, d=D, n_comp=10)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), cost_p=PEXP)
    return P, X, Y, cl


def test_cost_matrix_sampled(setup):
    P, X, Y, cl = setup
    rows = np.random.default_rng(1).choice(N, 64, replace=False)
    Cg = cl.cost_matrix().cpu().numpy()[rows].astype(np.float64)
    Cr = pcost.cost_matrix_p(X[rows], Y, PEXP)
    assert np.abs(Cg - Cr).max() <= 6e-6 * np.abs(Cr).max()


def test_half_steps_sampled(setup):
    """f' = f-update(g) at 256 sampled rows, g' = g-update(f') at 256 sampled
    columns, each against the FP64 soft-min over the whole other side."""
    P, X, Y, cl = setup
    eps = float(np.float32(cl.mean_cost / 20.0 / 16))
    f, g, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=30)
    f2, g2, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=1, g_init=g)
    g64 = g.cpu().numpy().astype(np.float64)
    f2_64 = f2.cpu().numpy().astype(np.float64)
    g2_64 = g2.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(13)
    rows = rng.choice(N, 256, replace=False)
    cols = rng.choice(M, 256, replace=False)
    ref_f = eps * np.log(1.0 / N) - eps * softmin_rows(pcost.cost_matrix_p(X[rows], Y, PEXP), g64, eps)
    ref_g = eps * np.log(1.0 / M) - eps * softmin_rows(pcost.cost_matrix_p(Y[cols], X, PEXP), f2_64, eps)
    ef = np.abs(f2_64[rows] - ref_f).max() / max(np.abs(f2_64).max(), eps)
    eg = np.abs(g2_64[cols] - ref_g).max() / max(np.abs(g2_64).max(), eps)
    print(f"full-size general cost half-steps: f {ef:.2e} g {eg:.2e}", flush=True)
    assert ef < 1e-4 and eg < 1e-4


def test_progot_last_step_sampled(setup):
    """The benchmark's ProgOT solve: its last potentials satisfy the g-update
    of the returned f at sampled columns (computed exactly by the oracle on
    the GPU's X^(K-1)), the FP64 marginal meets tau, and the final map at
    sampled points matches the oracle's map of X^(K-1)."""
    P, X, Y, cl = setup
    f, G, TX, info = P.progot_solve(cl, 4, theta=2.0 ** -4, tau_first=1e-3, tau_last=1e-3,
                                    max_iter=100_000)
    print(f"full-size general cost ProgOT: iters {info.iters}", flush=True)
    assert info.converged
    eps = float(np.float32(info.eps[-1]))
    xl = cl.xk().cpu().numpy()
    f64 = f.cpu().numpy().astype(np.float64)
    g64 = G[-1].cpu().numpy().astype(np.float64)
    cols = np.random.default_rng(14).choice(M, 128, replace=False)
    ref_g = eps * np.log(1.0 / M) - eps * softmin_rows(pcost.cost_matrix_p(Y[cols], xl, PEXP), f64, eps)
    eg = np.abs(g64[cols] - ref_g).max() / max(np.abs(g64).max(), eps)
    assert eg < 1e-4, eg
    row, col, _ = P.marginal_check(cl, f, G[-1], eps)
    assert row <= 1e-3 * 1.01 and col <= 1e-4
    pts = np.random.default_rng(15).choice(N, 64, replace=False)
    ref_t = pcost.entropic_map_p(xl[pts], Y, G[-1].cpu().numpy(), eps, PEXP)
    assert map_err(TX.cpu().numpy()[pts], ref_t, Y) < 1e-3
