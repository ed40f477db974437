"""The BF16 forms against the FP64 oracle.

BF16X3 (hi/lo split, three BF16 products) must meet the same bars as FP32
(potentials 1e-4, maps 1e-3).  Plain BF16 (one product, inputs rounded to 8
mantissa bits) is measured and reported per result on the precision
workload's 4096 x 4096 subsample, with a sanity bound only: its cross-term
error ~2^-9 |x| |y| / sqrt(d) is what the form trades for speed."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import pot_err, map_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    return P


@pytest.mark.parametrize("n,m,d", [(256, 256, 4), (1000, 777, 64), (300, 513, 100), (200, 700, 256),
                                   (1, 9, 7),
                                   # n << m: > 32 column splits, the last ones empty
                                   (130, 40000, 64)])
def test_bf16x3_fixed_iterations(P, n, m, d):
    X, Y = workloads.sphere(seed=200 + d, n=n, m=m, d=d, n_clusters=6)
    a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
    eps = float(np.float32(oracle.mean_cost(X, Y) / 20.0))
    print(f"case bf16x3 n={n} m={m} d={d}", flush=True)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision="bf16x3")
    for it in (1, 11):
        f, g, info = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=it)
        ref = oracle.sinkhorn(a, X, b, Y, eps, 0.0, n_iter=it)
        ef, eg = pot_err(f.cpu().numpy(), ref.f, eps), pot_err(g.cpu().numpy(), ref.g, eps)
        assert ef < 1e-4 and eg < 1e-4, (it, ef, eg)
    Q = workloads.sphere(seed=300 + d, n=min(n, 64), m=2, d=d, n_clusters=6)[0]
    g32 = g.cpu().numpy()
    for alpha in (1.0, 0.4):
        out = P.entropic_map(cl, g, eps, P.to_device(Q), alpha=alpha)
        ref_t = oracle.entropic_map(Q, Y, g32.astype(np.float64), eps, alpha=alpha)
        assert map_err(out.cpu().numpy(), ref_t, Y) < 1e-3


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("n,m,d", [(1000, 777, 64), (300, 513, 100), (200, 700, 256),
                                   # n << m: > 32 column splits, the last ones empty
                                   (130, 40000, 64)])
def test_fixed_shift_and_its_fallback(P, monkeypatch, prec, n, m, d):
    """From the second iteration the BF16 partial kernels shift each row by
    the log-sum-exp of its previous potential instead of a running maximum.
    With PROGOT_BF16_SHIFT=recheck every fixed-shift sweep fails its range
    check and is redone with the running maximum: the same bits as =off
    (running maximum only).  The default (fixed shift) agrees with both to
    FP32 rounding of the exponents, and BF16X3 meets the oracle bar."""
    X, Y = workloads.sphere(seed=500 + d, n=n, m=m, d=d, n_clusters=6)
    a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
    eps = float(np.float32(oracle.mean_cost(X, Y) / 20.0))
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    res = {}
    for mode in ("off", "recheck", "auto"):
        print(f"case {prec} n={n} m={m} d={d} shift={mode}", flush=True)
        if mode == "auto":
            monkeypatch.delenv("PROGOT_BF16_SHIFT", raising=False)
        else:
            monkeypatch.setenv("PROGOT_BF16_SHIFT", mode)
        f, g, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=11)
        res[mode] = (f.cpu().numpy(), g.cpu().numpy())
    monkeypatch.delenv("PROGOT_BF16_SHIFT", raising=False)
    assert np.array_equal(res["recheck"][0], res["off"][0])
    assert np.array_equal(res["recheck"][1], res["off"][1])
    for k in (0, 1):
        assert pot_err(res["auto"][k], res["off"][k], eps) < 1e-5
    if prec == "bf16x3":
        ref = oracle.sinkhorn(a, X, b, Y, eps, 0.0, n_iter=11)
        assert pot_err(res["auto"][0], ref.f, eps) < 1e-4 and pot_err(res["auto"][1], ref.g, eps) < 1e-4


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
def test_progot_warm_start_shift(P, monkeypatch, prec):
    """From the second ProgOT step the first iteration's exponent shift comes
    from the warm start, (1 - alpha_k) times the previous step's potentials.
    Over a whole solve PROGOT_BF16_SHIFT=recheck (every fixed-shift sweep
    redone with the running maximum) reproduces =off bit for bit, and the
    default meets the ProgOT bars against the oracle (BF16X3)."""
    n, m, d = 1500, 1200, 64
    X, Y = workloads.sphere(seed=640, n=n, m=m, d=d, n_clusters=6)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    res = {}
    for mode in ("off", "recheck", "auto"):
        print(f"case ProgOT {prec} n={n} m={m} d={d} shift={mode}", flush=True)
        if mode == "auto":
            monkeypatch.delenv("PROGOT_BF16_SHIFT", raising=False)
        else:
            monkeypatch.setenv("PROGOT_BF16_SHIFT", mode)
        f, G, TX, info = P.progot_solve(cl, 4, tau_first=1e-3, tau_last=1e-3)
        res[mode] = (f.cpu().numpy(), G.cpu().numpy(), TX.cpu().numpy(), list(info.iters))
    monkeypatch.delenv("PROGOT_BF16_SHIFT", raising=False)
    for k in range(3):
        assert np.array_equal(res["recheck"][k], res["off"][k])
    assert res["recheck"][3] == res["off"][3]
    if prec == "bf16x3":
        a, b = np.full(n, 1.0 / n), np.full(m, 1.0 / m)
        ref = oracle.progot(a, X, b, Y, 4, tau=1e-3)
        assert all(abs(p - q) <= 2 for p, q in zip(res["auto"][3], ref.iters))
        assert map_err(res["auto"][2], ref.TX, Y) < 1e-3


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("nq,m,d", [(300, 1000, 128), (333, 999, 200), (129, 1025, 256), (1, 33, 256),
                                    # 128- and 64-column map tiles (d <= 64), the last one ragged
                                    (257, 777, 20), (200, 1000, 64), (65, 130, 48)])
def test_bf16_map_ragged(P, prec, nq, m, d):
    """Entropic map of both BF16 forms on ragged sizes (query blocks and the
    last column tile partly filled; d = 200 pads to 256, d = 20 and 48 to
    32 and 64, where the tiles are 64 or 128 columns wide) against FP64, at
    a converged target potential.  BF16X3 meets the 1e-3 map bar; plain BF16
    (weights and cross term rounded once) is held to a sanity bound, 5e-3 at
    d >= 128 and 1e-2 at d <= 64: there eps (mean cost/20) is small against
    the clusters' internal spread, so a few columns carry each row's weight
    and their ~2^-8 relative cross-term errors average out less (the same
    error with 32-column tiles, 7.7e-3 at d = 20)."""
    X, Y = workloads.sphere(seed=400 + d, n=max(nq, 64), m=m, d=d, n_clusters=5)
    Q = X[:nq]
    eps = float(np.float32(oracle.mean_cost(X, Y) / 20.0))
    print(f"case map {prec} nq={nq} m={m} d={d}", flush=True)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    f, g, _ = P.sinkhorn_solve(cl, eps, tau=1e-3)
    g64 = g.cpu().numpy().astype(np.float64)
    for alpha in (1.0, 0.3):
        out = P.entropic_map(cl, g, eps, P.to_device(Q), alpha=alpha)
        ref = oracle.entropic_map(Q, Y, g64, eps, alpha=alpha)
        e = map_err(out.cpu().numpy(), ref, Y)
        print(f"  alpha {alpha}: map err {e:.2e}", flush=True)
        assert e < (1e-3 if prec == "bf16x3" else 5e-3 if d > 64 else 1e-2)


@pytest.mark.parametrize("prec", ["bf16x3", "bf16"])
@pytest.mark.parametrize("nq,m,d", [(257, 1, 128), (7, 1, 256), (100, 65, 100), (300, 65, 256),
                                    (129, 33, 128), (513, 97, 200), (70, 129, 128), (33, 200, 256)])
def test_map_tile_counts(P, prec, nq, m, d):
    """The BF16 maps at d = 128 and 256 (warp-specialised) run the weights of
    column tile t one interval after its scores, in pairs of intervals with
    one left over for an odd tile count: one tile (m = 1, the left-over
    interval alone), two (a pair), three (a pair and the left-over one), on
    ragged query counts; tiles are 32 columns (BF16X3) or 64 (plain BF16).
    For m = 1 the map is the single target point whatever the potential, so
    that case takes a zero potential instead of a solve.  Bars as in
    test_bf16_map_ragged."""
    X, Y = workloads.sphere(seed=500 + d + m, n=max(nq, 64), m=m, d=d, n_clusters=3)
    Q = X[:nq]
    eps = float(np.float32(max(oracle.mean_cost(X, Y), 1e-3) / 20.0))
    print(f"case {prec} map nq={nq} m={m} d={d}", flush=True)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    if m == 1:
        g = torch.zeros(1, dtype=torch.float32, device="cuda")
    else:
        _, g, _ = P.sinkhorn_solve(cl, eps, tau=1e-3)
    g64 = g.cpu().numpy().astype(np.float64)
    for alpha in (1.0, 0.3):
        out = P.entropic_map(cl, g, eps, P.to_device(Q), alpha=alpha)
        ref = oracle.entropic_map(Q, Y, g64, eps, alpha=alpha)
        e = map_err(out.cpu().numpy(), ref, Y)
        print(f"  alpha {alpha}: map err {e:.2e}", flush=True)
        assert e < (1e-3 if prec == "bf16x3" else 5e-3)


def test_precision_table(P):
    """The precision workload's protocol on its seeded 4096 x 4096 subsample
    (d = 256, 32 unit-norm clusters + N(0, 0.01 I)): Sinkhorn at mean cost/20
    for a fixed 30 iterations, then the entropic map of the sources; errors
    of FP32, BF16X3 and BF16 against FP64."""
    X, Y = workloads.sphere(seed=3, n=65536, m=65536, d=256, n_clusters=32)
    idx = workloads.subsample_index(65536, 4096, seed=33)
    Xs, Ys = X[idx], Y[idx]
    n = 4096
    a = np.full(n, 1.0 / n)
    eps = float(np.float32(oracle.mean_cost(Xs, Ys) / 20.0))
    ref = oracle.sinkhorn(a, Xs, a, Ys, eps, 0.0, n_iter=30)
    ref_t = oracle.entropic_map(Xs, Ys, ref.g, eps)
    rows = {}
    for prec in ("fp32", "bf16x3", "bf16"):
        cl = P.prepare_clouds(P.to_device(Xs), P.to_device(Ys), precision=prec)
        f, g, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=30)
        T = P.entropic_map(cl, g, eps, P.to_device(Xs))
        # map of the oracle's potential isolates the map kernel's own error
        T_ref_g = P.entropic_map(cl, P.to_device(ref.g.astype(np.float32)), eps, P.to_device(Xs))
        rows[prec] = (pot_err(f.cpu().numpy(), ref.f, eps), pot_err(g.cpu().numpy(), ref.g, eps),
                      map_err(T.cpu().numpy(), ref_t, Ys), map_err(T_ref_g.cpu().numpy(), ref_t, Ys))
    print("precision table (4096 subsample, d=256): form  f_err  g_err  map_err  map_err(oracle g)")
    for k, v in rows.items():
        print(f"  {k:7s} " + "  ".join(f"{x:.2e}" for x in v), flush=True)
    for k in ("fp32", "bf16x3"):
        assert rows[k][0] < 1e-4 and rows[k][1] < 1e-4 and rows[k][2] < 1e-3 and rows[k][3] < 1e-3
    assert max(rows["bf16"]) < 5e-2


def test_progot_bf16x3_c1(P):
    X, Y = workloads.c1(seed=1)
    n = X.shape[0]
    a = np.full(n, 1.0 / n)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision="bf16x3")
    f, G, TX, info = P.progot_solve(cl, 4, tau_first=1e-3, tau_last=1e-3)
    ref = oracle.progot(a, X, a, Y, 4, tau=1e-3)
    assert info.converged
    assert all(abs(p - q) <= 2 for p, q in zip(info.iters, ref.iters))
    assert map_err(TX.cpu().numpy(), ref.TX, Y) < 1e-3
    row, col, _ = P.marginal_check(cl, f, G[-1], info.eps[-1])
    assert row <= 1e-3 * 1.01 and col <= 1e-4


def test_bf16x3_small_eps_limit_is_a_warning(P):
    """The form's limit at small eps, recorded: ProgOT (K = 4) on the small
    workload's clouds at n = m = 4096, d = 16 with eps_k = 0.03 mean cost/20.
    The late steps' potentials are ~1e4 eps, so BF16X3's ~2^-16 relative
    cross-term error is an absolute exponent error near tau: its marginal
    error stalls above tau = 1e-3 and the solve returns
    POT_WARN_NOT_CONVERGED with finite outputs, where FP32 (2^-24) meets tau
    in every step."""
    X, Y = workloads.c1(seed=7, n=4096, m=4096, d=16)
    res = {}
    for prec in ("fp32", "bf16x3"):
        print(f"case ProgOT {prec} c1 4096 d=16 theta=0.03", flush=True)
        cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
        f, G, TX, info = P.progot_solve(cl, 4, theta=0.03, max_iter=3000)
        assert torch.isfinite(f).all() and torch.isfinite(G).all() and torch.isfinite(TX).all()
        res[prec] = info
        print(f"  status {info.status} iters {info.iters} err {info.err}", flush=True)
    assert res["fp32"].status == 0 and res["fp32"].converged
    assert res["bf16x3"].status == P.progot.POT_WARN_NOT_CONVERGED
    assert max(res["bf16x3"].err) > 1e-3 and max(res["bf16x3"].err) < 1e-2
