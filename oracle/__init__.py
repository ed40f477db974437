"""FP64 CPU oracle for progressive entropic optimal transport (ProgOT).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path
(no kernels, headers, helpers or constants); the two meet only through the
seeded inputs of ``workloads``.

Everything here is plain NumPy in float64 on a *materialised* cost matrix
C_ij = sum_k (x_ik - y_jk)^2 computed by direct differences (deliberately not
the |x|^2 + |y|^2 - 2<x, y> expansion the GPU uses).  Inputs are the FP32
arrays the GPU receives, upcast to FP64.

Readings of the paper adopted here (garbled or silent passages):

* cost h = |.|^2 (no 1/2), as in the experiments (Sec. 5); eps is always
  set relative to the mean cost, so the 1/2 of the theory (Sec. 3.2) is the
  same problem at eps/2 and the map is identical.
* coupling P_ij = exp((f_i + g_j - C_ij)/eps) with P 1 = a and P^T 1 = b:
  the only sign-consistent reading of the dual (eq. entdual) and of the
  Sinkhorn algorithm (Alg. 1), whose printed signs are inconsistent.
* Alg. 1 updates read f <- eps log a + min_eps(C - f (+) g) + f, i.e.
  f_i = eps log a_i - eps LSE_j((g_j - C_ij)/eps), and the symmetric g-update.
* Alg. 1 loops *while* the row-marginal L1 error exceeds tau (the printed
  "<" cannot be the loop condition); the error is checked after each full
  (f, g) iteration and that (f, g) is returned.
* entropic map T(x) = sum_j softmax_j((g_j - |x - y_j|^2)/eps) y_j with no
  b_j factor: this equals the row-normalised coupling of Alg. 2 at training
  points; Alg. 3's b_j factor belongs to the convention where the weights
  sit outside the potentials and cancels for uniform b.
* K counts Sinkhorn solves, k = 0..K-1; constant speed is alpha_k = 1/(K-k)
  (the t-column of the alpha-schedule table is self-consistent, its alpha
  column is off by one).
* warm start (Alg. 2) scales the previous potentials by (1 - alpha_k), as
  printed; a switch selects (1 - alpha_{k-1}).
* a stopped-at-max_iter solve is reported, not fatal ("infinite iteration
  budget" in Sec. 5.2 is not runnable).
* general costs (``pcost``): h = (1/p)|.|_p^p, the form of Sec. 5.2 and of
  the map appendix (whose "1.5 |.|_1.5" is read as this h with p = 1.5);
  potentials keep the convention above and the per-step eps rule uses the
  mean of h over all pairs.

Parity pins for every function are in ``tests/test_oracle_*.py``.
"""
from .sinkhorn import (cost_matrix, sinkhorn, SinkhornResult, coupling, marginal_errors,
                       dual_objective, primal_objective, mean_cost)
from .entropic_map import entropic_map, map_weights
from .progot import progot, progot_map, ProgOTResult
from . import schedules
from . import metrics
from . import pcost

__all__ = [
    "cost_matrix", "sinkhorn", "SinkhornResult", "coupling", "marginal_errors",
    "dual_objective", "primal_objective", "mean_cost", "entropic_map", "map_weights",
    "progot", "progot_map", "ProgOTResult", "schedules", "metrics", "pcost",
]
