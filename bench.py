#!/usr/bin/env python
"""ProgOT benchmark on one MI355X.

A step is one full ProgOT solve (Alg. 2) on device-resident clouds: per-step
eps from the mean cost, K warm-started Sinkhorn solves to tau = 1e-3 (fused
cost + log-sum-exp kernels), the McCann-type moves between them and the final
map X^(K).  Workload (default): n = m = 16384, d = 64, two independent
10-component Gaussian mixtures (centres ~ N(0, 9 I), std ~ U[0.5, 2]),
uniform weights, plain FP32, K = 8 constant speed, eps_k = mean cost / 20.

Prints one JSON line (stdout).  value = sum_k n m iters_k / solve time.
The roofline entry is for the dominant kernel (the fused cost + LSE
partial kernel): algorithmic flops per launch = 2 n m d (the cross term of
every pair) over its average launch time, measured with HIP events on the
stream it runs on.  cpu_baseline is the FP64 oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

METRIC = "ProgOT solve time @ marginal err 1e-3; n·m·iters/s; serve p50/p99 latency"
PEAK = {"fp32": 157.3, "bf16": 2500.0}   # TFLOP/s, dense MFMA, MI355X
PAD = {16: 16, 64: 64, 128: 128, 256: 256}  # template dimension of the kernel per d
QB = {16: 2, 64: 2, 128: 2, 256: 1}

WORKLOADS = {
    # name: (generator kwargs, K, precision)
    "gmm16k_d64_fp32": (dict(kind="gmm", seed=2, n=16384, m=16384, d=64), 8, "fp32"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_clouds(spec):
    kind = spec["kind"]
    kw = {k: v for k, v in spec.items() if k != "kind"}
    if kind == "gmm":
        return workloads.gmm(**kw)
    if kind == "sphere":
        return workloads.sphere(**kw)
    raise ValueError(kind)


def recorded_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 --pmc record, or None
    when there is none or the kernel source changed since it was taken."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2406_05061_amd", "csrc", "progot_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    if rec.get("kernel_sha256_16") != sha or rec.get("workload") != workload:
        return None
    return float(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def cpu_baseline(X, Y, n_sample: int, max_iter: int):
    """FP64 oracle (as it stands) on the first n_sample points of a seeded
    permutation of each cloud: one Sinkhorn solve at eps = mean cost / 20,
    tau = 1e-3, bounded to max_iter iterations."""
    import importlib
    import oracle
    osk = importlib.import_module("oracle.sinkhorn")
    idx = workloads.subsample_index(X.shape[0], n_sample, seed=33)
    idy = workloads.subsample_index(Y.shape[0], n_sample, seed=34)
    Xs, Ys = X[idx], Y[idy]
    a = np.full(n_sample, 1.0 / n_sample)
    t0 = time.perf_counter()
    eps = oracle.mean_cost(Xs, Ys) / 20.0
    r = oracle.sinkhorn(a, Xs, a, Ys, eps, 1e-3, max_iter=max_iter)
    dt = time.perf_counter() - t0
    return {"value": n_sample * n_sample * r.iters / dt, "unit": "n·m·iters/s",
            "cores": osk.THREADS, "kind": "oracle",
            "sample": f"FP64 oracle Sinkhorn on a {n_sample}x{n_sample} seeded subsample of the "
                      f"same clouds, eps = mean cost/20, tau 1e-3, {r.iters} iterations "
                      f"(max {max_iter}), cost matrix build included, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gmm16k_d64_fp32", choices=sorted(WORKLOADS))
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--cpu-iters", type=int, default=20)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to scale "
                         "hardware byte counters, and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU only: this build has no multi-GPU path "
            "(run with --gpus 1).")
        sys.exit(2)

    import torch
    import paper_2406_05061_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"bench: copied {nbytes} bytes 3 times")
        return
    spec, K, prec = WORKLOADS[args.workload]
    X, Y = make_clouds(spec)
    n, d = X.shape
    m = Y.shape[0]
    log(f"bench: {args.workload}: n={n} m={m} d={d} K={K} {prec} tau={args.tau}")
    Xd, Yd = P.to_device(X), P.to_device(Y)
    cl = P.prepare_clouds(Xd, Yd, precision=prec)

    def step():
        return P.progot_solve(cl, K, tau_first=args.tau, tau_last=args.tau)

    for w in range(args.warmup):
        _, _, _, info = step()
        log(f"bench: warmup {w}: iters {info.iters} in {info.seconds:.3f} s")
    torch.cuda.synchronize()

    P.timing_enable(True)
    iters_total = 0
    infos = []
    t0 = time.perf_counter()
    for s in range(args.steps):
        f, G, TX, info = step()
        iters_total += sum(info.iters)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lse_ms, lse_n, map_ms, map_n = P.timing_read()
    P.timing_enable(False)
    elapsed = t1 - t0
    log(f"bench: {args.steps} solves in {elapsed:.3f} s; iters per solve {infos[-1].iters}")

    row, col, dual = P.marginal_check(cl, f, G[-1], infos[-1].eps[-1])
    log(f"bench: final FP64 marginal L1 row {row:.3e} col {col:.3e}")

    value = n * m * iters_total / elapsed
    avg_lse_s = lse_ms * 1e-3 / max(lse_n, 1)
    flops = 2.0 * n * m * d
    achieved = flops / avg_lse_s / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "n·m·iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "K": K,
                   "precision": prec, "tau": args.tau, "eps": "mean cost/20 per step",
                   "alpha": "constant speed"},
        "solve_time_s": elapsed / args.steps,
        "sinkhorn_iters_per_solve": infos[-1].iters,
        "final_marginal_l1_fp64": {"row": row, "col": col},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[prec],
                     "traffic": recorded_traffic(f"lse_partial_{prec}<{PAD[d]},{QB[d]}>",
                                                 args.workload),
                     "kernel": "lse_partial (fused cost + log-sum-exp)",
                     "avg_launch_us": avg_lse_s * 1e6, "launches": lse_n,
                     "flops_per_launch": flops},
        "map_kernel": {"avg_launch_us": map_ms * 1e3 / max(map_n, 1), "launches": map_n},
    }
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle, {args.cpu_sample}^2 sample) ...")
        out["cpu_baseline"] = cpu_baseline(X, Y, args.cpu_sample, args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
