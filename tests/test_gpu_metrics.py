"""Evaluation metrics on the GPU (FP64 coupling pass, diagonal pass,
Sinkhorn divergence) against the oracle's."""
import numpy as np
import pytest

import oracle
from oracle import metrics
from oracle.sinkhorn import cost_matrix
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    return P


@pytest.mark.parametrize("n,m,d,weighted", [(700, 500, 16, True), (257, 1031, 64, False), (1, 33, 5, False)])
def test_coupling_metrics_match_oracle(P, n, m, d, weighted):
    """Same (f, g) on both sides: every metric is an FP64 sum of the same
    terms (the GPU forms C with an FP64 MFMA cross term, the oracle by
    direct differences), so they agree to ~1e-9 relative."""
    X, Y = workloads.gmm(seed=40 + d, n=n, m=m, d=d)
    a = workloads.weights(n, seed=41) if weighted else None
    b = workloads.weights(m, seed=42) if weighted else None
    print(f"case metrics n={n} m={m} d={d} weighted={weighted}", flush=True)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), a=None if a is None else P.to_device(a),
                          b=None if b is None else P.to_device(b))
    eps = float(np.float32(oracle.mean_cost(X, Y) / 20.0))
    f, g, _ = P.sinkhorn_solve(cl, eps, tau=1e-4)
    met = P.coupling_metrics(cl, f, g, eps)
    # the FP32 weights as the GPU reads them (not renormalised in FP64)
    aa = np.full(n, 1.0 / n) if a is None else a.astype(np.float64)
    bb = np.full(m, 1.0 / m) if b is None else b.astype(np.float64)
    C = cost_matrix(X, Y)
    f64, g64 = f.cpu().numpy().astype(np.float64), g.cpu().numpy().astype(np.float64)
    Pm = oracle.coupling(f64, g64, C, eps)
    row, col = oracle.marginal_errors(f64, g64, C, eps, aa, bb)
    ref = {"transport_cost": metrics.transport_cost(Pm, C), "p_log_p": metrics.p_log_p(Pm),
           "mass": float(Pm.sum()), "ot": oracle.dual_objective(f64, g64, C, eps, aa, bb)}
    for k, v in ref.items():
        assert abs(met[k] - v) <= 1e-9 * max(abs(v), 1.0), (k, met[k], v)
    assert abs(met["row_err"] - row) <= 1e-9 + 1e-6 * row
    assert abs(met["col_err"] - col) <= 1e-9 + 1e-6 * col


def test_diag_metrics_spd(P):
    """Trace and KL of the coupling-recovery benchmark on an SPD pair."""
    X, Y = workloads.spd_pair(seed=9, n=512, d=6)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
    C = cost_matrix(X, Y)
    for beta in (1.0, 0.1):
        eps = float(np.float32(beta * C.mean() / 20.0))
        f, g, _ = P.sinkhorn_solve(cl, eps, tau=1e-4)
        tr, kl = P.diag_metrics(cl, f, g, eps)
        ref_tr, ref_kl = metrics.diag_metrics(oracle.coupling(f.cpu().numpy(), g.cpu().numpy(), C, eps))
        print(f"beta {beta}: Tr {tr:.6f} KL {kl:.6f}", flush=True)
        assert abs(tr - ref_tr) <= 1e-9 * ref_tr and abs(kl - ref_kl) <= 1e-9 * max(1.0, abs(ref_kl))
    assert tr > 0.95
    with pytest.raises(P.PotError):
        cl2 = P.prepare_clouds(P.to_device(X), P.to_device(Y[:100]))
        P.diag_metrics(cl2, f[:512], g[:100], eps)


def test_sinkhorn_divergence_matches_oracle(P):
    """Default eps_D (5 % of the mean cost within Y) and an explicit eps; both
    sides stop by Alg. 1's rule at tau = 1e-5 (near the FP32 floor of the
    marginal error), so the objectives agree to O(eps tau).  (The oracle's
    values at tau = 1e-5 and 1e-6 differ by <= 1.4e-5 here, against the
    1e-4 eps bar; 1e-6 took ten times as long.)"""
    X, Y = workloads.gmm(seed=50, n=600, m=500, d=8)
    for eps in (0.0, None):
        out = P.sinkhorn_divergence(P.to_device(X), P.to_device(Y), eps=0.0 if eps == 0.0 else 2.0,
                                    tau=1e-5)
        e = out["eps"]
        ref = metrics.sinkhorn_divergence(np.full(600, 1 / 600), X, np.full(500, 1 / 500), Y, eps=e,
                                          tau=1e-5)
        print(f"eps {e:.4f}: D gpu {out['D']:.6f} oracle {ref[0]:.6f}", flush=True)
        if eps == 0.0:
            assert abs(e - metrics.eps_divergence_default(Y)) <= 1e-6 * e
        assert out["status"] == 0
        for k, v in zip(("D", "ot_xy", "ot_xx", "ot_yy"), ref[:4]):
            assert abs(out[k] - v) <= 1e-4 * e + 1e-5 * abs(v), (k, out[k], v)


def test_sinkhorn_divergence_translation(P):
    """D(X, X + t) = |t|^2 for equal uniform weights (exact identity; X on a
    2^-10 grid so X + t is exact in FP32)."""
    X = (np.round(workloads.gmm(seed=51, n=1000, m=10, d=8)[0] * 1024) / 1024).astype(np.float32)
    t = np.array([0.5, -0.25, 1.0, 0.0, 0.125, -1.5, 0.75, 0.25], dtype=np.float32)
    Y = (X + t).astype(np.float32)
    tt = float((t.astype(np.float64) ** 2).sum())
    mc = oracle.mean_cost(X, X)
    out = P.sinkhorn_divergence(P.to_device(X), P.to_device(Y), eps=float(0.5 * mc), tau=1e-5)
    print(f"translation: D {out['D']:.6f} |t|^2 {tt:.6f}", flush=True)
    assert abs(out["D"] - tt) <= 1e-4 * tt + 1e-4 * out["eps"]
