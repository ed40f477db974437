"""Serving form: requests of uneven (n, m, d) advanced together by the server
(grouped kernels, admission by arena footprint, requests joining between
ticks) produce the same bits as each solve run alone, and the alone result
is itself parity-tested against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import workloads
from tests.parity import map_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SIZES = [(300, 500, 16), (1000, 777, 64), (2048, 1536, 128), (257, 3000, 64), (4096, 256, 16),
         (5000, 4500, 64), (64, 64, 128)]


@pytest.fixture(scope="module")
def P():
    assert torch.cuda.is_available()
    import paper_2406_05061_amd as P
    return P


def _clouds(i, n, m, d):
    return workloads.gmm(seed=4_000_000 + i, n=n, m=m, d=d)


def test_server_equals_alone_with_queueing(P):
    K = 3
    reqs = []
    for i, (n, m, d) in enumerate(SIZES):
        X, Y = _clouds(i, n, m, d)
        reqs.append((P.to_device(X), P.to_device(Y)))
    alone = []
    for X, Y in reqs:
        cl = P.prepare_clouds(X, Y)
        f, G, TX, info = P.progot_solve(cl, K, tau_first=1e-3, tau_last=1e-3)
        alone.append((f, G, TX, info))
    # arena for ~3 of the larger requests: later ones wait for space
    per = max(P.Server.request_bytes(n, m, d) for n, m, d in SIZES)
    srv = P.Server(3 * per + (1 << 20), max_active=4)
    pending = list(range(len(reqs)))
    rid_of, out = {}, {}
    ticks = 0
    while pending or rid_of:
        # two requests first, the rest join while others are mid-solve
        room = 2 if ticks < 3 else len(pending)
        admitted = []
        for i in pending[:room]:
            rid = srv.submit(reqs[i][0], reqs[i][1], K, tau_first=1e-3, tau_last=1e-3)
            if rid is None:
                break
            rid_of[i] = rid
            admitted.append(i)
        pending = [i for i in pending if i not in admitted]
        srv.step()
        ticks += 1
        for i, rid in list(rid_of.items()):
            r = srv.poll(rid)
            if r is not None:
                out[i] = r
                del rid_of[i]
        assert ticks < 100_000
    srv.close()
    print(f"serving: {len(reqs)} requests in {ticks} ticks", flush=True)
    for i in range(len(reqs)):
        f, G, TX, info = out[i]
        fa, Ga, TXa, infoa = alone[i]
        assert info.iters == infoa.iters, (i, info.iters, infoa.iters)
        assert info.eps == infoa.eps
        assert torch.equal(f, fa) and torch.equal(G, Ga) and torch.equal(TX, TXa), i


def test_server_request_matches_oracle(P):
    X, Y = workloads.gmm(seed=77, n=700, m=600, d=16, n_comp=4)
    one = P.Server.request_bytes(700, 600, 16)
    srv = P.Server(P.Server.arena_overhead(2) + one + one // 2, max_active=2)
    rid = srv.submit(P.to_device(X), P.to_device(Y), 3, tau_first=1e-3, tau_last=1e-3)
    assert rid is not None
    # a second request cannot fit the arena now
    assert srv.submit(P.to_device(X), P.to_device(Y), 3) is None
    res = None
    while res is None:
        srv.step()
        res = srv.poll(rid)
    srv.close()
    f, G, TX, info = res
    ref = oracle.progot(np.full(700, 1 / 700), X, np.full(600, 1 / 600), Y, 3, tau=1e-3)
    assert all(abs(p - q) <= 2 for p, q in zip(info.iters, ref.iters))
    assert map_err(TX.cpu().numpy(), ref.TX, Y) < 1e-3
