"""Seeded synthetic point clouds for the progressive entropic OT hot path.

This module is the only code shared by the FP64 oracle tests and the GPU
path: it draws inputs and nothing else.  It holds none of the method's
arithmetic (no cost, no potential, no map).  Every generator draws in FP64
with ``numpy.random.default_rng(seed)`` (PCG64) and returns FP32 arrays, so
both sides of a parity test consume the very same FP32 values (the oracle
upcasts them to FP64).

The paper evaluates on single-cell data (sci-Plex, 4i), CIFAR-10 and a
Gaussian-mixture benchmark, none of which is available here.  The shapes
below bracket those workloads (Sec. 5: n of order 1e3..6e4, d from 4 to
1024) and stand in for them.

Recipes (variance is written as ``N(mean, var)``):

* ``c1``      -- X: n points ~ N(0, I_d); Y: m points from a 4-component
                 mixture, centres ~ N(0, 4 I), covariances A A^T + 0.1 I with
                 A entries ~ N(0, 0.5), labels uniform.
* ``gmm``     -- each cloud an independent mixture of ``n_comp`` isotropic
                 Gaussians, centres ~ N(0, 9 I), per-component std ~ U[0.5, 2].
* ``sphere``  -- each cloud has ``n_clusters`` unit-norm centres v/|v|,
                 v ~ N(0, I), independent centre sets for source and target;
                 points are centre + N(0, 0.01 I).
* ``spd_pair``-- X ~ N(0, I), Y = X G^T with G symmetric positive definite
                 (the optimal matching is the identity, Prop. on the blurred
                 CIFAR benchmark, Sec. 5.3).
* ``request_stream`` -- the serving workload: Poisson arrivals, n and m
                 log-uniform in [256, 32768], d in {16, 64, 128}, gmm clouds.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _f32(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def c1(seed: int = 1, n: int = 1024, m: int = 1024, d: int = 4, n_comp: int = 4):
    """Source N(0, I) versus a 4-component Gaussian mixture target."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    mu = rng.standard_normal((n_comp, d)) * 2.0          # N(0, 4 I)
    A = rng.standard_normal((n_comp, d, d)) * math.sqrt(0.5)
    cov = A @ np.transpose(A, (0, 2, 1)) + 0.1 * np.eye(d)
    chol = np.linalg.cholesky(cov)
    lab = rng.integers(n_comp, size=m)
    z = rng.standard_normal((m, d))
    Y = mu[lab] + np.einsum("nij,nj->ni", chol[lab], z)
    return _f32(X), _f32(Y)


def c1_holdout(seed: int = 1, n: int = 1024, d: int = 4, n_comp: int = 4, m_test: int = 1024,
               test_seed: int = 101):
    """Fresh draws from the target mixture of c1(seed, n, ...) (same centres
    and covariances; labels and noise from test_seed): the hold-out targets
    of the eps-scheduler."""
    rng = np.random.default_rng(seed)
    rng.standard_normal((n, d))                          # the sources of c1
    mu = rng.standard_normal((n_comp, d)) * 2.0
    A = rng.standard_normal((n_comp, d, d)) * math.sqrt(0.5)
    cov = A @ np.transpose(A, (0, 2, 1)) + 0.1 * np.eye(d)
    chol = np.linalg.cholesky(cov)
    rt = np.random.default_rng(test_seed)
    lab = rt.integers(n_comp, size=m_test)
    z = rt.standard_normal((m_test, d))
    return _f32(mu[lab] + np.einsum("nij,nj->ni", chol[lab], z))


def _gmm_cloud(rng, n, d, n_comp):
    mu = rng.standard_normal((n_comp, d)) * 3.0          # N(0, 9 I)
    sd = rng.uniform(0.5, 2.0, size=n_comp)
    lab = rng.integers(n_comp, size=n)
    return mu[lab] + sd[lab, None] * rng.standard_normal((n, d))


def gmm(seed: int = 2, n: int = 16384, m: int = 16384, d: int = 64, n_comp: int = 10):
    """Two independent isotropic Gaussian mixtures (source, target)."""
    rng = np.random.default_rng(seed)
    X = _gmm_cloud(rng, n, d, n_comp)
    Y = _gmm_cloud(rng, m, d, n_comp)
    return _f32(X), _f32(Y)


def _sphere_centres(rng, k, d):
    v = rng.standard_normal((k, d))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _sphere_points(rng, centres, n):
    lab = rng.integers(centres.shape[0], size=n)
    return centres[lab] + 0.1 * rng.standard_normal((n, centres.shape[1]))


def sphere(seed: int = 3, n: int = 65536, m: int = 65536, d: int = 256,
           n_clusters: int = 32, n_query: int = 0, query_seed: int = 55):
    """Clustered unit-norm clouds; optional out-of-sample queries drawn from the
    source distribution (same centres, separate seed)."""
    rng = np.random.default_rng(seed)
    cx = _sphere_centres(rng, n_clusters, d)
    cy = _sphere_centres(rng, n_clusters, d)
    X = _sphere_points(rng, cx, n)
    Y = _sphere_points(rng, cy, m)
    if n_query:
        Q = _sphere_points(np.random.default_rng(query_seed), cx, n_query)
        return _f32(X), _f32(Y), _f32(Q)
    return _f32(X), _f32(Y)


def spd_pair(seed: int = 7, n: int = 256, d: int = 8, cond: float = 4.0):
    """X ~ N(0, I) and Y = X G^T, G symmetric positive definite with
    eigenvalues log-spaced in [1, cond]."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, d))
    Qm, _ = np.linalg.qr(rng.standard_normal((d, d)))
    G = (Qm * np.geomspace(1.0, cond, d)) @ Qm.T
    return _f32(X), _f32(X @ G.T)


def weights(n: int, seed: int | None = None, spread: float = 0.5):
    """Uniform weights (seed None) or a seeded positive probability vector with
    entries in [(1-spread)/n, (1+spread)/n] before normalisation."""
    if seed is None:
        return np.full(n, 1.0 / n, dtype=np.float32)
    rng = np.random.default_rng(seed)
    w = rng.uniform(1.0 - spread, 1.0 + spread, size=n)
    w = w / w.sum()
    return w.astype(np.float32)


def subsample_index(n: int, k: int, seed: int = 33):
    """First k entries of a seeded permutation of range(n)."""
    return np.random.default_rng(seed).permutation(n)[:k]


@dataclass
class Request:
    rid: int
    arrival_s: float
    n: int
    m: int
    d: int
    seed: int


def request_stream(n_req: int = 2048, qps: float = 100.0, seed: int = 4,
                   n_lo: int = 256, n_hi: int = 32768, dims=(16, 64, 128)):
    """Poisson arrivals; n and m independently log-uniform in [n_lo, n_hi];
    d uniform over ``dims``.  Clouds of request r come from ``gmm`` with seed
    4e6 + r (drawn lazily by the caller)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=n_req)
    t = np.cumsum(gaps) - gaps[0]
    lo, hi = math.log(n_lo), math.log(n_hi)
    ns = np.round(np.exp(rng.uniform(lo, hi, size=n_req))).astype(int)
    ms = np.round(np.exp(rng.uniform(lo, hi, size=n_req))).astype(int)
    ds = rng.choice(np.asarray(dims), size=n_req)
    return [Request(r, float(t[r]), int(ns[r]), int(ms[r]), int(ds[r]), 4_000_000 + r)
            for r in range(n_req)]


def request_clouds(req: Request):
    return gmm(seed=req.seed, n=req.n, m=req.m, d=req.d)
