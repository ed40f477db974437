"""Failure paths of the C ABI, driven by ordinary arithmetic (no fault): a NaN
or infinity in the clouds or in an initial potential makes the mean cost or
the marginal error non-finite, which every entry point reports as
POT_ERR_NUMERIC; the serving form retires only the failing request; a solve
that runs out of iterations returns POT_WARN_NOT_CONVERGED with finite
outputs."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    return P


def _pair(seed=91, n=600, m=500, d=16):
    return workloads.gmm(seed=seed, n=n, m=m, d=d, n_comp=4)


@pytest.mark.parametrize("bad", [np.nan, np.inf])
@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_prepare_reports_non_finite_clouds(P, bad, prec):
    X, Y = _pair()
    X[17, 3] = bad
    print(f"case prepare with {bad} in X, {prec}", flush=True)
    with pytest.raises(P.PotError) as e:
        P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    assert e.value.code == P.progot.POT_ERR_NUMERIC


def test_progot_solve_reports_nan_source(P):
    """The clouds were prepared from finite X; X then gets a NaN (the caller's
    input, which Alg. 2 reads again when it resets the source iterate)."""
    X, Y = _pair()
    Xd = P.to_device(X)
    cl = P.prepare_clouds(Xd, P.to_device(Y))
    Xd[5, 0] = float("nan")
    print("case progot_solve with NaN in X", flush=True)
    with pytest.raises(P.PotError) as e:
        P.progot_solve(cl, 3)
    assert e.value.code == P.progot.POT_ERR_NUMERIC


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_sinkhorn_reports_nan_potential(P, prec):
    X, Y = _pair(n=900, m=1100, d=64)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=prec)
    g0 = torch.zeros(Y.shape[0], dtype=torch.float32, device="cuda")
    g0[123] = float("nan")
    eps = cl.mean_cost / 20
    print(f"case sinkhorn_solve with a NaN initial potential, {prec}", flush=True)
    for tau in (1e-3, 0.0):     # tolerance mode and fixed-iteration mode
        with pytest.raises(P.PotError) as e:
            P.sinkhorn_solve(cl, eps, tau=tau, max_iter=5, g_init=g0)
        assert e.value.code == P.progot.POT_ERR_NUMERIC
    # the same clouds still solve afterwards
    f, g, info = P.sinkhorn_solve(cl, eps, tau=1e-3)
    assert info.status == 0 and torch.isfinite(f).all() and torch.isfinite(g).all()


def test_max_iter_is_a_warning_with_finite_outputs(P):
    X, Y = _pair()
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
    eps = cl.mean_cost / 20
    f, g, info = P.sinkhorn_solve(cl, eps, tau=1e-7, max_iter=3)
    assert info.status == P.progot.POT_WARN_NOT_CONVERGED and not info.converged
    assert info.iters == 3 and np.isfinite(info.err) and info.err > 1e-7
    assert torch.isfinite(f).all() and torch.isfinite(g).all()
    f2, G, TX, pinfo = P.progot_solve(cl, 2, tau_first=1e-7, tau_last=1e-7, max_iter=4)
    assert pinfo.status == P.progot.POT_WARN_NOT_CONVERGED and not pinfo.converged
    assert pinfo.iters == [4, 4]
    assert torch.isfinite(G).all() and torch.isfinite(TX).all()


def test_server_retires_only_the_failing_request(P):
    """A request whose source cloud holds a NaN finishes with
    POT_ERR_NUMERIC; every other request of the mix, before and after it,
    gets the same bits as when solved alone, and the loop never raises."""
    K = 3
    sizes = [(700, 600, 16), (1500, 1300, 64), (900, 1000, 16), (400, 2100, 128)]
    reqs = []
    for i, (n, m, d) in enumerate(sizes):
        X, Y = workloads.gmm(seed=5_000_000 + i, n=n, m=m, d=d)
        reqs.append((P.to_device(X), P.to_device(Y)))
    alone = [P.progot_solve(P.prepare_clouds(X, Y), K) for X, Y in reqs]
    bad_X, bad_Y = workloads.gmm(seed=5_000_100, n=800, m=700, d=64)
    bad_X[400, 7] = np.nan
    bad = (P.to_device(bad_X), P.to_device(bad_Y))
    order = [reqs[0], reqs[1], bad, reqs[2], reqs[3]]
    srv = P.Server(sum(P.Server.request_bytes(X.shape[0], Y.shape[0], X.shape[1])
                       for X, Y in order) + (4 << 20), max_active=8)
    print("case server with one NaN request among four", flush=True)
    rids = [srv.submit(X, Y, K) for X, Y in order]
    assert all(r is not None for r in rids)
    results, failed = {}, {}
    ticks = 0
    while len(results) + len(failed) < len(order):
        srv.step()
        ticks += 1
        for j, rid in enumerate(rids):
            if j in results or j in failed:
                continue
            try:
                r = srv.poll(rid)
            except P.PotError as e:
                failed[j] = e.code
                continue
            if r is not None:
                results[j] = r
        assert ticks < 100_000
    assert failed == {2: P.progot.POT_ERR_NUMERIC}
    assert not srv.live            # the failed request's tensors were dropped too
    srv.close()
    for j, i in zip([0, 1, 3, 4], range(4)):
        f, G, TX, info = results[j]
        fa, Ga, TXa, infoa = alone[i]
        assert info.iters == infoa.iters
        assert torch.equal(f, fa) and torch.equal(G, Ga) and torch.equal(TX, TXa), i
