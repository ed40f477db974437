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
# TFLOP/s of the cross term, dense MFMA, MI355X: FP32; BF16; BF16X3 runs three
# BF16 products per algorithmic product, so its ceiling is the BF16 peak / 3.
PEAK = {"fp32": 157.3, "bf16": 2500.0, "bf16x3": 2500.0 / 3}
PAD = {16: 16, 64: 64, 128: 128, 256: 256}  # template dimension of the kernel per d
QB = {16: 4, 64: 4, 128: 2, 256: 1}

_SPHERE64K = dict(kind="sphere", seed=3, n=65536, m=65536, d=256, n_clusters=32)
_SPHERE256K = dict(kind="sphere", seed=5, n=262144, m=262144, d=128, n_clusters=64,
                   n_query=1 << 20, query_seed=55)
WORKLOADS = {
    # name: (generator kwargs, K, precision)
    "gmm16k_d64_fp32": (dict(kind="gmm", seed=2, n=16384, m=16384, d=64), 8, "fp32"),
    # precision workload: 32 unit-norm clusters + N(0, 0.01 I), d = 256
    "sphere64k_d256_fp32": (_SPHERE64K, 4, "fp32"),
    "sphere64k_d256_bf16": (_SPHERE64K, 4, "bf16"),
    "sphere64k_d256_bf16x3": (_SPHERE64K, 4, "bf16x3"),
    # large map estimation: fit on 64 unit-norm clusters, then T_Prog on 2^20
    # queries drawn from the source distribution
    "sphere256k_d128_bf16": (_SPHERE256K, 8, "bf16"),
    "sphere256k_d128_bf16x3": (_SPHERE256K, 8, "bf16x3"),
    # the same in FP32, the baseline of the BF16 forms' speedup
    "sphere256k_d128_fp32": (_SPHERE256K, 8, "fp32"),
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


# What the FP32 potential kernel is built from: its source, the headers it
# includes and the build flags.
KERNEL_SOURCES = ["paper_2406_05061_amd/csrc/progot_kernels.hip",
                  "paper_2406_05061_amd/csrc/progot_device.h",
                  "paper_2406_05061_amd/csrc/progot_internal.h",
                  "paper_2406_05061_amd/build.py"]


# ... and the general-cost potential kernels.
PCOST_SOURCES = ["paper_2406_05061_amd/csrc/progot_pcost.hip",
                 "paper_2406_05061_amd/csrc/progot_device.h",
                 "paper_2406_05061_amd/csrc/progot_internal.h",
                 "paper_2406_05061_amd/build.py"]


def kernel_source_sha(sources=None) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in (KERNEL_SOURCES if sources is None else sources):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, sources=None):
    """HBM bytes per launch from the committed rocprofv3 --pmc record, or None
    when there is none or the kernel source changed since it was taken."""
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
    except (OSError, KeyError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != kernel_source_sha(sources) or rec.get("workload") != workload:
        return None
    return float(rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"])


def cpu_model() -> str:
    """The host CPU's model name (first processor of /proc/cpuinfo)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(X, Y, n_sample: int, n_iter: int):
    """FP64 oracle (as it stands) on the first n_sample points of a seeded
    permutation of each cloud: the first n_iter iterations of a Sinkhorn
    solve at eps = mean cost / 20 (fixed-iteration mode, so the sample is a
    bounded ~10 s of CPU work however fast the solve converges)."""
    import importlib
    import oracle
    osk = importlib.import_module("oracle.sinkhorn")
    idx = workloads.subsample_index(X.shape[0], n_sample, seed=33)
    idy = workloads.subsample_index(Y.shape[0], n_sample, seed=34)
    Xs, Ys = X[idx], Y[idy]
    a = np.full(n_sample, 1.0 / n_sample)
    t0 = time.perf_counter()
    eps = oracle.mean_cost(Xs, Ys) / 20.0
    r = oracle.sinkhorn(a, Xs, a, Ys, eps, 0.0, n_iter=n_iter)
    dt = time.perf_counter() - t0
    return {"value": n_sample * n_sample * r.iters / dt, "unit": "n·m·iters/s",
            "cores": osk.THREADS, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"FP64 oracle Sinkhorn on a {n_sample}x{n_sample} seeded subsample of the "
                      f"same clouds, eps = mean cost/20, {r.iters} fixed iterations, cost matrix "
                      f"build included, {dt:.1f} s"}


def serve_bench(args):
    """Serving workload: a Poisson stream of ProgOT solves (K = 4) with n, m
    log-uniform in [256, 32768] and d in {16, 64, 128}.  (1) closed loop:
    every request submitted at once -> saturation solves/s; (2) open loop at
    0.7 x saturation, latency = finish - scheduled arrival; (3) the same
    arrivals served first-in first-out by single pot_progot_solve calls."""
    import torch
    import paper_2406_05061_amd as P

    K, tau = 4, args.tau
    reqs = workloads.request_stream(n_req=args.requests, qps=1.0, seed=4)
    log(f"bench: serve: {len(reqs)} requests, K={K}, generating clouds")
    data = []
    for r in reqs:
        X, Y = workloads.request_clouds(r)
        data.append((P.to_device(X), P.to_device(Y)))
    torch.cuda.synchronize()
    pair_flops = [2.0 * r.n * r.m * r.d for r in reqs]
    arena = args.arena_gib << 30

    def run_server(arrivals):
        srv = P.Server(arena, max_active=args.max_active)
        t0 = time.perf_counter()
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        pending, rid_of, done = 0, {}, {}
        infos = {}
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while pending < len(order) and arrivals[order[pending]] <= now:
                i = order[pending]
                rid = srv.submit(data[i][0], data[i][1], K, tau_first=tau, tau_last=tau,
                                 want_TX=True)
                if rid is None:
                    break
                rid_of[rid] = i
                pending += 1
            if rid_of:
                srv.step()
                now = time.perf_counter() - t0
                for rid, i in list(rid_of.items()):
                    res = srv.poll(rid)
                    if res is not None:
                        done[i] = now
                        infos[i] = res[3]
                        del rid_of[rid]
                        if len(done) % 256 == 0:
                            log(f"bench: serve: {len(done)} of {len(reqs)} done at {now:.1f} s")
            elif pending < len(order):
                time.sleep(max(0.0, min(0.01, arrivals[order[pending]] - now)))
        wall = time.perf_counter() - t0
        srv.close()
        return wall, done, infos

    def lat_stats(done, arrivals):
        lat = np.array([done[i] - arrivals[i] for i in range(len(reqs))])
        return float(np.percentile(lat, 50) * 1e3), float(np.percentile(lat, 99) * 1e3)

    # (1) saturation
    zero = [0.0] * len(reqs)
    P.timing_enable(True)
    wall_sat, done_sat, infos_sat = run_server(zero)
    lse_ms, lse_n, _, _ = P.timing_read()
    P.timing_enable(False)
    sat = len(reqs) / wall_sat
    flops = sum(pair_flops[i] * 2 * sum(it + 1 for it in infos_sat[i].iters)
                for i in range(len(reqs)))
    log(f"bench: serve saturation {sat:.2f} solves/s ({wall_sat:.1f} s)")
    # (2) open loop at 0.7 x saturation
    qps = 0.7 * sat
    rng = np.random.default_rng(4)
    gaps = rng.exponential(1.0 / qps, size=len(reqs))
    arrivals = list(np.cumsum(gaps) - gaps[0])
    wall_srv, done_srv, infos_srv = run_server(arrivals)
    p50, p99 = lat_stats(done_srv, arrivals)
    log(f"bench: serve open loop qps {qps:.2f}: p50 {p50:.1f} ms p99 {p99:.1f} ms")
    # (3) FIFO baseline with single solves
    t0 = time.perf_counter()
    done_seq = {}
    for i in sorted(range(len(reqs)), key=lambda i: arrivals[i]):
        now = time.perf_counter() - t0
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        cl = P.prepare_clouds(data[i][0], data[i][1])
        P.progot_solve(cl, K, tau_first=tau, tau_last=tau)
        done_seq[i] = time.perf_counter() - t0
        if len(done_seq) % 256 == 0:
            log(f"bench: FIFO: {len(done_seq)} of {len(reqs)} done at {done_seq[i]:.1f} s")
    wall_seq = time.perf_counter() - t0
    b50, b99 = lat_stats(done_seq, arrivals)
    log(f"bench: FIFO single solves: p50 {b50:.1f} ms p99 {b99:.1f} ms ({wall_seq:.1f} s)")
    achieved = flops / (lse_ms * 1e-3) / 1e12 if lse_ms > 0 else 0.0
    out = {
        "metric": METRIC, "value": len(reqs) / wall_srv, "unit": "solves/s", "n_gpus": 1,
        "steps": len(reqs), "warmup": 0, "ms_per_step": wall_srv / len(reqs) * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serve", "requests": len(reqs), "K": K, "tau": tau,
                   "n_m": "log-uniform [256, 32768]", "d": [16, 64, 128],
                   "qps": qps, "max_active": args.max_active, "arena_gib": args.arena_gib},
        "latency_ms": {"p50": p50, "p99": p99},
        "saturation_solves_per_s": sat,
        "fifo_single_solve": {"solves_per_s": len(reqs) / wall_seq, "p50_ms": b50, "p99_ms": b99},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK["fp32"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK["fp32"], "traffic": None,
                     "kernel": "lse_partial grouped (saturation run)", "launches": lse_n},
    }
    print(json.dumps(out), flush=True)


NEXT_WORKLOADS = ("alg4_c1", "divergence_gmm16k", "pcost_4i_d47")
# The cost h = (1/p)|.|_p^p, p = 1.5, at the shape of the paper's coupling
# experiment on single-cell data (about 11000 control and 2800 treated cells,
# 47 features), K = 4 constant speed, eps_k = 2^-4 mean cost / 20, tau 1e-3:
# two 10-component Gaussian mixtures stand in for the cells.
_PCOST = dict(kind="gmm", seed=12, n=11000, m=2800, d=47, n_comp=10)
HBM_PEAK_GBS = 8000.0
# The library times launches 0, 15, 30, ... of each kernel inside the timed
# region (odd, so f- and g-updates are sampled alike): timing every launch
# costs two events and their host bookkeeping per launch, which slowed the
# 23 us general-cost updates' solve by ~18 % and the benchmark's by ~2 %.
TIMING_EVERY = 15


def timing_every_for(n: int, m: int, d: int) -> int:
    """Every launch is timed where launches take milliseconds (n m d >= 2^36:
    the precision and large-map workloads), so that the few updates of a
    step that differ from the rest (the first, without an exponent shift in
    the BF16 forms) are not over- or under-sampled; every 15th elsewhere."""
    return 1 if n * m * d >= 1 << 36 else TIMING_EVERY


def next_bench(args):
    """Steps beyond the ProgOT solve, each timed beside the FP64 oracle:
    alg4_c1 -- Alg. 4 (eps-scheduler, 7 grid scales) on the small ProgOT
    workload (n = m = 1024, d = 4, 1024 hold-out targets), against the
    oracle's Alg. 4 on the same problem; divergence_gmm16k -- the Sinkhorn
    divergence (eq. sink_div, eps_D default, tau 1e-3) of the benchmark's
    clouds (16384^2, d = 64), against the oracle on a 2048^2 subsample."""
    import torch
    import paper_2406_05061_amd as P
    import oracle
    from oracle import metrics
    osk = __import__("importlib").import_module("oracle.sinkhorn")

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        P.timing_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        lse_ms, lse_n, _, _ = P.timing_read()
        P.timing_enable(False)
        return r, dt, lse_ms / reps, lse_n // reps

    out = {"metric": METRIC, "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    if args.workload == "pcost_4i_d47":
        pcost_bench(args, out)
        return
    if args.workload == "alg4_c1":
        X, Y = workloads.c1(seed=1)
        Yt = workloads.c1_holdout(seed=1, test_seed=101)
        K, tau = 4, args.tau
        cl = P.prepare_clouds(P.to_device(X), P.to_device(Y))
        Ytd = P.to_device(Yt)
        sched, dt, lse_ms, lse_n = timed(lambda: P.eps_schedule(cl, Ytd, K, tau=tau), args.steps)
        log(f"bench: alg4_c1: {dt * 1e3:.1f} ms per schedule, p* {sched.p_star}, "
            f"{lse_n} potential launches")
        a = np.full(1024, 1.0 / 1024)
        t0 = time.perf_counter()
        ref, info = oracle.schedules.eps_scheduler(a, X, a, Y, oracle.schedules.alpha_schedule(K), Yt,
                                                    beta0=5.0, tau=tau)
        t_cpu = time.perf_counter() - t0
        out.update({"value": dt * 1e3, "unit": "ms per schedule", "ms_per_step": dt * 1e3,
                    "config": {"workload": "alg4_c1", "n": 1024, "m": 1024, "d": 4, "K": K,
                               "grid": "2^-3..2^3", "m_test": 1024, "tau": tau},
                    "p_star": sched.p_star, "oracle_p_star": info["p_star"],
                    "eps": sched.eps, "potential_launches": lse_n,
                    "potential_kernel_ms": lse_ms,
                    "cpu_baseline": {"value": t_cpu * 1e3, "unit": "ms per schedule",
                                     "cores": osk.THREADS, "cpu_model": cpu_model(), "kind": "oracle",
                                     "sample": "the full problem (FP64 oracle Alg. 4, 7 grid solves "
                                               "of 1024 x 1024, hold-out maps)"}})
    else:
        X, Y = make_clouds(WORKLOADS["gmm16k_d64_fp32"][0])
        Xd, Yd = P.to_device(X), P.to_device(Y)
        res, dt, lse_ms, lse_n = timed(lambda: P.sinkhorn_divergence(Xd, Yd, tau=args.tau), args.steps)
        n, d = X.shape
        flops = 2.0 * n * n * d * lse_n
        log(f"bench: divergence_gmm16k: D {res['D']:.6g} eps {res['eps']:.4g} in {dt * 1e3:.1f} ms, "
            f"{lse_n} potential launches")
        idx = workloads.subsample_index(n, 2048, seed=33)
        idy = workloads.subsample_index(n, 2048, seed=34)
        a = np.full(2048, 1.0 / 2048)
        t0 = time.perf_counter()
        refD = metrics.sinkhorn_divergence(a, X[idx], a, Y[idy], eps=res["eps"], tau=args.tau)
        t_cpu = time.perf_counter() - t0
        out.update({"value": dt * 1e3, "unit": "ms per divergence", "ms_per_step": dt * 1e3,
                    "config": {"workload": "divergence_gmm16k", "n": n, "m": n, "d": d,
                               "eps": "5% of the mean cost within Y", "tau": args.tau},
                    "D": res["D"], "eps_D": res["eps"], "potential_launches": lse_n,
                    "roofline": {"bound": "mfma", "achieved": flops / (lse_ms * 1e-3) / 1e12,
                                 "peak": PEAK["fp32"], "unit": "TFLOP/s",
                                 "frac": flops / (lse_ms * 1e-3) / 1e12 / PEAK["fp32"],
                                 "traffic": None, "kernel": "lse_partial (fused cost + log-sum-exp)"},
                    "cpu_baseline": {"value": t_cpu * 1e3, "unit": "ms per divergence",
                                     "cores": osk.THREADS, "cpu_model": cpu_model(), "kind": "oracle",
                                     "sample": f"FP64 oracle divergence on a 2048 x 2048 seeded "
                                               f"subsample (D = {refD[0]:.6g}), same eps_D and tau"}})
    print(json.dumps(out), flush=True)


def pcost_bench(args, out):
    """ProgOT with h = (1/p)|.|_p^p, p = 1.5 (Sec. 5.2's second cost).  A step
    is one ProgOT solve: per step the cost matrix of (X^(k), Y) is built once
    (VALU), each Sinkhorn half-iteration streams it (row or column
    log-sum-exp), and the McCann step runs the fused p-cost map.  The
    roofline is the potential kernels' HBM bound: algorithmic bytes per
    launch = n m 4 (the cost matrix read once) over the average launch."""
    import torch
    import paper_2406_05061_amd as P
    from oracle import pcost
    osk = __import__("importlib").import_module("oracle.sinkhorn")
    p, K, theta, tau = 1.5, 4, 2.0 ** -4, args.tau
    X, Y = make_clouds(_PCOST)
    n, d = X.shape
    m = Y.shape[0]
    log(f"bench: pcost_4i_d47: n={n} m={m} d={d} p={p} K={K} theta={theta} tau={tau}")
    cl = P.prepare_clouds(P.to_device(X), P.to_device(Y), cost_p=p, cost_mode=args.cost_mode)

    def step():
        # run to convergence, as the coupling experiment does; the last solve
        # starts cold (the printed warm start scales by 1 - alpha_{K-1} = 0)
        return P.progot_solve(cl, K, theta=theta, tau_first=tau, tau_last=tau,
                              max_iter=args.max_iter)

    _, _, _, info = step()
    log(f"bench: warmup: iters {info.iters} in {info.seconds:.3f} s")
    torch.cuda.synchronize()
    P.timing_enable(True, every=TIMING_EVERY)
    iters_total, infos = 0, []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        f, G, TX, info = step()
        iters_total += sum(info.iters)
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    lse_ms, lse_n, map_ms, map_n = P.timing_read()
    P.timing_enable(False)
    row, col, _ = P.marginal_check(cl, f, G[-1], infos[-1].eps[-1])
    avg_lse = lse_ms * 1e-3 / max(lse_n, 1)
    gbs = n * m * 4 / avg_lse / 1e9
    log(f"bench: {args.steps} solves in {elapsed:.3f} s; iters {infos[-1].iters}; potential launch "
        f"{avg_lse * 1e6:.1f} us = {gbs:.0f} GB/s; FP64 marginal L1 row {row:.3e} col {col:.3e}")
    out.update({"value": n * m * iters_total / elapsed, "unit": "n·m·iters/s", "higher_is_better": True,
                "ms_per_step": elapsed / args.steps * 1e3, "solve_time_s": elapsed / args.steps,
                "config": {"workload": "pcost_4i_d47", "n": n, "m": m, "d": d, "cost": "(1/p)|.|_p^p",
                           "p": p, "K": K, "theta": theta, "tau": tau, "alpha": "constant speed",
                           "cost_matrix": "kept" if cl.c.cmat else "on the fly"},
                "sinkhorn_iters_per_solve": infos[-1].iters,
                "final_marginal_l1_fp64": {"row": row, "col": col},
                "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": gbs / HBM_PEAK_GBS,
                             "traffic": recorded_traffic("pcost_lse", "pcost_4i_d47", PCOST_SOURCES),
                             "kernel": "pcost_lse_rows / pcost_lse_cols (resident cost matrix)",
                             "avg_launch_us": avg_lse * 1e6, "timed_launches": lse_n,
                             "timing_every": TIMING_EVERY,
                             "bytes_per_launch": n * m * 4},
                "map_kernel": {"avg_launch_us": map_ms * 1e3 / max(map_n, 1), "timed_launches": map_n}})
    if not args.no_cpu_baseline:
        ns, ms, it = 2048, 512, 100
        idx = workloads.subsample_index(n, ns, seed=33)
        idy = workloads.subsample_index(m, ms, seed=34)
        t0 = time.perf_counter()
        Cs = pcost.cost_matrix_p(X[idx], Y[idy], p)
        r = osk.sinkhorn(np.full(ns, 1.0 / ns), X[idx], np.full(ms, 1.0 / ms), Y[idy],
                         theta * Cs.mean() / 20.0, tau, max_iter=it, C=Cs)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": ns * ms * r.iters / dt, "unit": "n·m·iters/s", "cores": osk.THREADS,
            "kind": "oracle",
            "sample": f"FP64 oracle Sinkhorn for the same cost on a {ns}x{ms} seeded subsample, "
                      f"eps = 2^-4 mean cost/20, tau {tau}, {r.iters} iterations (max {it}), cost "
                      f"matrix build included, {dt:.1f} s"}
    print(json.dumps(out), flush=True)


FORMS = ("fp32", "bf16", "bf16x3")


def forms_bench(args) -> dict:
    """The precision workload (n = m = 65536, d = 256, 32 unit-norm clusters +
    N(0, 0.01 I), K = 4, eps_k = mean cost/20, tau) solved by ProgOT in each
    arithmetic form of the cross term, timed the same way as the main line:
    solve time, Sinkhorn iterations, the FP64 row/column marginal L1 of the
    returned coupling (the equal-error condition of the speed-ups) and the
    potential kernel's fraction of its MFMA peak (every launch timed; they
    last milliseconds)."""
    import torch
    import paper_2406_05061_amd as P
    spec, K = _SPHERE64K, 4
    X, Y = make_clouds(spec)
    n, d = X.shape
    m = Y.shape[0]
    log(f"bench: forms: precision workload n={n} m={m} d={d} K={K}")
    Xd, Yd = P.to_device(X), P.to_device(Y)
    res = {"workload": "sphere64k_d256", "n": n, "m": m, "d": d, "K": K, "tau": args.tau,
           "steps": args.forms_steps, "warmup": 1}
    for prec in FORMS:
        cl = P.prepare_clouds(Xd, Yd, precision=prec)

        def step():
            return P.progot_solve(cl, K, tau_first=args.tau, tau_last=args.tau)

        step()
        torch.cuda.synchronize()
        P.timing_enable(True, every=1)
        t0 = time.perf_counter()
        for _ in range(args.forms_steps):
            f, G, TX, info = step()
        torch.cuda.synchronize()
        solve_s = (time.perf_counter() - t0) / args.forms_steps
        lse_ms, lse_n, _, _ = P.timing_read()
        P.timing_enable(False)
        row, col, _ = P.marginal_check(cl, f, G[-1], info.eps[-1])
        avg = lse_ms * 1e-3 / max(lse_n, 1)
        achieved = 2.0 * n * m * d / avg / 1e12
        res[prec] = {"solve_s": solve_s, "sinkhorn_iters_per_solve": info.iters,
                     "final_marginal_l1_fp64": {"row": row, "col": col},
                     "meets_tau": bool(row <= args.tau * 1.01 and col <= args.tau * 1.01),
                     "roofline": {"kernel": "lse_partial", "bound": "mfma",
                                  "achieved": achieved, "peak": PEAK[prec], "unit": "TFLOP/s",
                                  "frac": achieved / PEAK[prec], "avg_launch_us": avg * 1e6,
                                  "timed_launches": lse_n}}
        log(f"bench: forms: {prec}: {solve_s * 1e3:.1f} ms per solve, iters {info.iters}, "
            f"FP64 marginal {row:.2e}/{col:.2e}, lse_partial {achieved:.1f} TFLOP/s "
            f"({achieved / PEAK[prec]:.2f} of peak)")
        del cl, f, G, TX
        torch.cuda.empty_cache()
    for prec in FORMS[1:]:
        res[prec]["speedup_vs_fp32"] = res["fp32"]["solve_s"] / res[prec]["solve_s"]
    return res


def probe_bench(args):
    """One short run of the hot kernels at a chosen shape, for profilers:
    seeded clouds (clustered unit-norm, or Gaussian mixtures with
    --gen gmm), --iters Sinkhorn iterations in fixed-iteration mode at
    eps = theta * mean cost / 20 (each one f- and one g-update), then --maps
    launches of the entropic map on the source cloud; --cost-p selects the
    cost (1/p)|.|_p^p.  Prints the wall times as one JSON line."""
    import torch
    import paper_2406_05061_amd as P
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
    print(json.dumps({"workload": "probe", "gen": args.gen, "n": args.n, "m": m, "d": args.d,
                      "precision": args.prec, "cost_p": args.cost_p, "theta": args.theta,
                      "iters": args.iters, "sinkhorn_s": t1 - t0, "maps": args.maps,
                      "maps_s": t2 - t1}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="gmm16k_d64_fp32",
                    choices=sorted(WORKLOADS) + ["serve", "probe", *NEXT_WORKLOADS])
    ap.add_argument("--requests", type=int, default=2048, help="serve: number of requests")
    ap.add_argument("--max-active", type=int, default=128, help="serve: server slots")
    ap.add_argument("--arena-gib", type=int, default=16, help="serve: HBM budget of the server")
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=100_000, help="pcost_4i_d47: per solve")
    ap.add_argument("--cost-mode", default="auto", choices=["auto", "keep", "on_the_fly"],
                    help="pcost_4i_d47: keep the cost matrix or form it in every update")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="default workload: skip the precision forms of the 65536^2 workload")
    ap.add_argument("--forms-steps", type=int, default=3, help="timed solves per precision form")
    g = ap.add_argument_group("probe workload (profiling driver)")
    g.add_argument("--gen", default="sphere", choices=["sphere", "gmm"])
    g.add_argument("--n", type=int, default=65536)
    g.add_argument("--m", type=int, default=0, help="target points (default n)")
    g.add_argument("--d", type=int, default=128)
    g.add_argument("--prec", default="bf16", choices=list(FORMS))
    g.add_argument("--cost-p", type=float, default=0.0)
    g.add_argument("--theta", type=float, default=1.0)
    g.add_argument("--iters", type=int, default=1)
    g.add_argument("--maps", type=int, default=1)
    g.add_argument("--seed", type=int, default=5)
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--cpu-iters", type=int, default=48,
                    help="oracle iterations of the CPU baseline sample")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to scale "
                         "hardware byte counters, and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        log("bench.py measures one GPU only: the library has no multi-GPU path "
            "(run with --gpus 1).")
        sys.exit(2)

    import torch
    import paper_2406_05061_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "serve":
        serve_bench(args)
        return
    if args.workload in NEXT_WORKLOADS:
        next_bench(args)
        return
    if args.workload == "probe":
        probe_bench(args)
        return
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
    Q = None
    if spec.get("n_query"):
        X, Y, Q = make_clouds(spec)
    else:
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

    every = timing_every_for(n, m, d)
    P.timing_enable(True, every=every)
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

    tc = time.perf_counter()
    row, col, dual = P.marginal_check(cl, f, G[-1], infos[-1].eps[-1])
    t_check = time.perf_counter() - tc
    log(f"bench: final FP64 marginal L1 row {row:.3e} col {col:.3e} ({t_check * 1e3:.1f} ms)")

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
        "dtype": {"fp32": "f32", "bf16": "bf16", "bf16x3": "bf16x3"}[prec],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "d": d, "K": K,
                   "precision": prec, "tau": args.tau, "eps": "mean cost/20 per step",
                   "alpha": "constant speed"},
        "solve_time_s": elapsed / args.steps,
        "sinkhorn_iters_per_solve": infos[-1].iters,
        "final_marginal_l1_fp64": {"row": row, "col": col, "check_seconds": t_check},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK[prec],
                     "unit": "TFLOP/s", "frac": achieved / PEAK[prec],
                     "traffic": recorded_traffic(f"lse_partial_{prec}<{PAD[d]},{QB[d]}>",
                                                 args.workload),
                     "kernel": "lse_partial (fused cost + log-sum-exp)",
                     "avg_launch_us": avg_lse_s * 1e6, "timed_launches": lse_n,
                     "timing_every": every, "flops_per_launch": flops},
        "map_kernel": {"avg_launch_us": map_ms * 1e3 / max(map_n, 1), "timed_launches": map_n},
    }
    if Q is not None:
        # out-of-sample progressive map (Alg. 3) of the fitted state
        Qd = P.to_device(Q)
        P.progot_map(cl, G, infos[-1].eps, infos[-1].alpha, Qd[:4096])   # warm-up
        torch.cuda.synchronize()
        P.timing_enable(True)
        t0 = time.perf_counter()
        Yq = P.progot_map(cl, G, infos[-1].eps, infos[-1].alpha, Qd)
        torch.cuda.synchronize()
        t_eval = time.perf_counter() - t0
        _, _, mms, mn = P.timing_read()
        P.timing_enable(False)
        nq = Q.shape[0]
        mflops = 4.0 * nq * m * d            # cross term + projection per step
        out["eval"] = {"queries": nq, "seconds": t_eval, "queries_per_s": nq / t_eval,
                       "map_avg_launch_us": mms * 1e3 / max(mn, 1), "launches": mn,
                       "map_tflops": mflops / (mms * 1e-3 / max(mn, 1)) / 1e12}
        log(f"bench: T_Prog on {nq} queries: {t_eval:.2f} s")
        del Yq
    if not args.no_cpu_baseline:
        log(f"bench: cpu baseline (oracle, {args.cpu_sample}^2 sample) ...")
        out["cpu_baseline"] = cpu_baseline(X, Y, args.cpu_sample, args.cpu_iters)
    if args.workload == "gmm16k_d64_fp32" and not args.no_forms:
        del cl, Xd, Yd, f, G, TX
        torch.cuda.empty_cache()
        out["forms"] = forms_bench(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
