"""One launch of each hot kernel at a chosen shape, for profilers.

    python -m paper_2406_05061_amd.kernel_probe --n 65536 --d 128 --prec bf16
    python -m paper_2406_05061_amd.kernel_probe --gen gmm --n 11000 --m 2800 --d 47 --cost-p 1.5 --theta 0.0625

Prepares two seeded clouds (clustered unit-norm, or Gaussian mixtures with
--gen gmm; n x d and m x d), runs `--iters` Sinkhorn iterations at eps =
theta * mean cost / 20 (each iteration is one f-update and one g-update of
the potential kernels) and `--maps` launches of the entropic-map kernel on
the source cloud, then prints the wall times.  --cost-p P selects the cost
(1/P)|.|_P^P instead of the squared-Euclidean one.  Every step runs in
libprogot.so; this file only drives it.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gen", default="sphere", choices=["sphere", "gmm"])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--m", type=int, default=0, help="target points (default n)")
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--cost-p", type=float, default=0.0)
    ap.add_argument("--cost-mode", default="auto", choices=["auto", "keep", "on_the_fly"],
                    help="general cost: keep the cost matrix or form it in every update")
    ap.add_argument("--theta", type=float, default=1.0)
    ap.add_argument("--prec", default="bf16", choices=["fp32", "bf16", "bf16x3"])
    ap.add_argument("--iters", type=int, default=1)
    ap.add_argument("--maps", type=int, default=1)
    ap.add_argument("--seed", type=int, default=5)
    args = ap.parse_args()

    import torch
    import paper_2406_05061_amd as P
    import workloads

    m = args.m or args.n
    if args.gen == "gmm":
        X, Y = workloads.gmm(seed=args.seed, n=args.n, m=m, d=args.d, n_comp=10)
    else:
        X, Y = workloads.sphere(seed=args.seed, n=args.n, m=m, d=args.d, n_clusters=64)
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), precision=args.prec, cost_p=args.cost_p,
                          cost_mode=args.cost_mode)
    eps = args.theta * cl.mean_cost / 20.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, g, _ = P.sinkhorn_solve(cl, eps, tau=0.0, max_iter=args.iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Xq = cl.xk()
    for _ in range(args.maps):
        P.entropic_map(cl, g, eps, Xq)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"kernel_probe n={args.n} m={m} d={args.d} {args.prec} cost_p={args.cost_p}: "
          f"{args.iters} Sinkhorn iterations "
          f"{t1 - t0:.4f} s, {args.maps} maps {t2 - t1:.4f} s", flush=True)


if __name__ == "__main__":
    main()
