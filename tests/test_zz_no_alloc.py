"""The allocation-free Sinkhorn divergence (pot_sinkhorn_divergence_noalloc):
its workspace is the library's static per-GPU scratch array.  Checked
against pot_sinkhorn_divergence (caller workspace) on the same inputs, for
two calls in a row with the second smaller, so the second call runs on the
scratch the first one left behind."""
import numpy as np
import pytest

import paper_2406_05061_amd as P
from paper_2406_05061_amd import progot as B
import workloads

pytestmark = pytest.mark.gpu


def _pair(seed, n, m, d):
    X, Y = workloads.gmm(seed=seed, n=n, m=m, d=d)
    return P.to_device(X), P.to_device(Y)


def test_noalloc_divergence_equals_workspace_divergence():
    import torch
    cases = [(61, 3000, 2500, 64), (62, 700, 900, 16)]
    for seed, n, m, d in cases:
        print(f"noalloc divergence: seed {seed} n={n} m={m} d={d}", flush=True)
        X, Y = _pair(seed, n, m, d)
        torch.cuda.synchronize()
        alloc_before = torch.cuda.memory_allocated()
        got = B.sinkhorn_divergence_noalloc(X, Y, tau=1e-4)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == alloc_before
        ref = P.sinkhorn_divergence(X, Y, tau=1e-4)
        assert got["status"] == ref["status"] == 0
        for key in ("D", "ot_xy", "ot_xx", "ot_yy", "eps"):
            # same kernels, same iterates, same returned iterate: same bits
            assert got[key] == ref[key], (key, got[key], ref[key])


def test_noalloc_weighted_and_repeated():
    import torch
    X, Y = _pair(63, 1200, 800, 32)
    rng = np.random.default_rng(5)
    a = rng.uniform(0.5, 1.5, 1200)
    b = rng.uniform(0.5, 1.5, 800)
    a, b = P.to_device(a / a.sum()), P.to_device(b / b.sum())
    print("noalloc divergence: weighted 1200 x 800, d = 32, twice", flush=True)
    first = B.sinkhorn_divergence_noalloc(X, Y, a, b, tau=1e-4)
    second = B.sinkhorn_divergence_noalloc(X, Y, a, b, tau=1e-4)
    ref = P.sinkhorn_divergence(X, Y, a, b, tau=1e-4)
    for key in ("D", "ot_xy", "ot_xx", "ot_yy"):
        assert first[key] == second[key] == ref[key], key
    torch.cuda.synchronize()


def test_noalloc_rejects_oversize_pairs():
    import torch
    n = 70000   # the divergence workspace of a 70000^2, d = 64 pair exceeds the scratch
    assert P.lib().pot_sinkhorn_divergence_bytes(n, n, 64) > B.STATIC_SCRATCH_BYTES
    X = torch.zeros((n, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(P.PotError) as e:
        B.sinkhorn_divergence_noalloc(X, X)
    assert e.value.code == B.POT_ERR_NOMEM
