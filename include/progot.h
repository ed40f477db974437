/*
 * progot.h -- C ABI of the MI355X (gfx950) progressive entropic OT hot path.
 *
 * The library computes, on one GPU, the steps of progressive entropic optimal
 * transport (ProgOT, Kassraie et al. 2024):
 *   - log-domain Sinkhorn between two weighted point clouds under the cost
 *     h(x - y) = |x - y|^2 (Alg. 1 "Sink"; the entropic dual, eq. entdual);
 *   - the entropic map / barycentric projection and the McCann-type step
 *     x <- (1 - alpha) x + alpha T(x) (eq. Tent; Alg. 2, projection lines);
 *   - ProgOT itself (Alg. 2) and the progressive map T_Prog (Alg. 3).
 *
 * Conventions (readings of the paper; the same in the FP64 oracle):
 *   coupling  P_ij = exp((f_i + g_j - C_ij)/eps),  P 1 = a,  P^T 1 = b
 *   f-update  f_i = eps log a_i - eps LSE_j((g_j - C_ij)/eps)
 *   g-update  g_j = eps log b_j - eps LSE_i((f_i - C_ij)/eps)
 *   stop rule after each full (f, g) iteration, when |P 1 - a|_1 <= tau;
 *             the (f, g) of that iteration is returned
 *   map       T(x) = sum_j softmax_j((g_j - |x - y_j|^2)/eps) y_j
 *   K         number of Sinkhorn solves, k = 0..K-1, constant speed
 *             alpha_k = 1/(K - k) (alpha_{K-1} = 1)
 *
 * Memory and ownership.  Every pointer named "device" is device memory owned
 * by the caller.  The library never allocates device memory: all scratch
 * lives in a caller-provided workspace of pot_workspace_bytes() bytes (the
 * one exception, pot_sinkhorn_divergence_noalloc, uses a static array of
 * POT_STATIC_SCRATCH_BYTES per GPU that comes with the library).  The
 * pot_clouds struct is a host POD owned by the caller, valid while its
 * workspace lives.  X, Y, a, b are never written.  Layouts are row-major:
 * a cloud of n points in R^d is n*d floats, point i at [i*d, (i+1)*d).
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Work is enqueued on it.  pot_prepare_clouds, pot_sinkhorn_solve,
 * pot_progot_solve and pot_marginal_check block the calling host thread
 * (convergence checks and scalar read-backs); pot_entropic_map and
 * pot_progot_map do not.
 *
 * Errors.  Arguments are validated on the host before any launch; invalid
 * arguments return POT_ERR_INVALID and enqueue nothing.  A positive status is
 * a warning with valid outputs.  No C++ exception crosses the ABI.
 *
 * Host-side state.  The library keeps three pieces of process state, none of
 * it device memory a caller must manage: a small pinned, device-mapped host
 * buffer per host thread into which the Sinkhorn loop's kernels store their
 * error sums (with the event marking the end of that thread's last solve);
 * the process-wide switch and event lists of pot_timing_*; and the per-device
 * address of pot_sinkhorn_divergence_noalloc's static scratch array.
 *
 * Shape of the interface.  The convergence read-back has no check_every
 * argument: the loop reads the error back with a lag it picks from the cost
 * of one iteration (a stream never waits on the host for cheap iterations,
 * and no update past convergence runs for expensive ones), and returns the
 * first iterate with err <= tau in every case.  Continuous batching is the
 * pot_server_* family (admission, ticks, polling) rather than a single
 * group-step call, because admission and the per-request ProgOT schedule need
 * state between ticks.
 */
#ifndef PROGOT_H
#define PROGOT_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define POT_API __attribute__((visibility("default")))
#else
#define POT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    POT_OK = 0,
    POT_WARN_NOT_CONVERGED = 1, /* stopped at max_iter with err > tau; outputs valid   */
    POT_BUSY = 2,               /* serving: not admitted now / still in flight; retry  */
    POT_ERR_INVALID = -1,       /* bad sizes, null pointers, eps <= 0, K out of range  */
    POT_ERR_NOMEM = -2,         /* workspace smaller than pot_workspace_bytes()        */
    POT_ERR_NUMERIC = -3,       /* a non-finite marginal error or mean cost was seen    */
    POT_ERR_DEVICE = -4         /* a HIP runtime call failed                           */
} pot_status;

/* Arithmetic of the cross term <x_i, y_j> of the cost.  FP32: FP32 MFMA with
 * FP32 accumulation.  BF16: BF16 MFMA on copies rounded to nearest even,
 * FP32 accumulation.  BF16X3: each value split as hi + lo (hi = bf16(x),
 * lo = bf16(x - hi)) and the cross term formed as hi*hi + hi*lo + lo*hi on
 * BF16 MFMA (~2^-16 relative).  The projection product of the entropic map
 * is FP16 weights times a scaled FP16 copy of Y in the BF16 form, and split
 * weights times split targets (three products) in BF16X3.  Norms, the
 * log-sum-exp, potentials and marginal errors stay FP32 in every form.
 * In the BF16 forms the potential kernels shift each row's exponents by the
 * log-sum-exp of its previous potential (from the second Sinkhorn iteration
 * on) and fall back to a running maximum where a sum leaves [2^-64, 2^64];
 * the environment variable PROGOT_BF16_SHIFT, read at every launch, selects
 * the running maximum only ("off") or makes every fallback run ("recheck",
 * the same bits as "off"). */
typedef enum { POT_PREC_FP32 = 0, POT_PREC_BF16 = 1, POT_PREC_BF16X3 = 2 } pot_precision;

#define POT_MAX_D 256      /* largest supported dimension d                    */
#define POT_MAX_K 64       /* largest number of ProgOT steps K                  */

/* Device-resident pair of clouds with their precomputed per-point data
 * (filled by pot_prepare_clouds; all pointers are views into the caller's
 * inputs and workspace). */
typedef struct pot_clouds {
    int64_t n, m;          /* source and target sizes                           */
    int32_t d, precision;  /* dimension, pot_precision                          */
    const float *X, *Y;    /* caller inputs (device), n*d and m*d               */
    const float *a, *b;    /* caller weights (device) or NULL for uniform       */
    float *xk;             /* current source iterate X^(k) (device, n*d)        */
    float *x_sqn, *y_sqn;  /* |x_i|^2, |y_j|^2 (device, FP32, from FP64 sums)   */
    float *log_a, *log_b;  /* log weights (device)                              */
    void *x_lp, *y_lp;     /* BF16 [hi | lo] copies of xk and Y (BF16 forms)   */
    void *yt_lp;           /* transposed BF16 [hi | lo] copy of Y (BF16 forms)  */
    double mean_cost;      /* (1/nm) sum_ij h(x_i - y_j) for the current xk     */
    void *ws;              /* workspace base (device)                           */
    size_t ws_bytes;
    float cost_p;          /* 0: h = |.|^2; p > 1: h = (1/p)|.|_p^p             */
    float *cmat;           /* cost_p > 0: C_ij = h(xk_i - y_j), n x ldc (device),
                              or NULL when the cost is formed on the fly       */
    int64_t ldc;           /* row stride of cmat (m rounded up to 4), or 0      */
} pot_clouds;

/* Bytes of device workspace pot_prepare_clouds needs for these sizes (the
 * same workspace serves every later call on the pair).  0 if invalid. */
POT_API size_t pot_workspace_bytes(int64_t n, int64_t m, int32_t d, int32_t precision);

/* Step "prepare" of the path: squared norms (FP64 sums rounded to FP32), log
 * weights, the working copy xk = X, BF16 copies in the BF16 form, and the
 * mean cost (1/nm) sum_ij |x_i - y_j|^2 that sets eps_0 (Alg. 4, first set
 * line) and the per-step eps (App. C).
 *   X (device, n*d), Y (device, m*d); a (device, n) / b (device, m) are
 *   probability weights, or NULL for uniform 1/n, 1/m.
 *   ws (device, ws_bytes >= pot_workspace_bytes) is owned by the caller.
 * Blocks until the mean cost is on the host.  1 <= d <= POT_MAX_D. */
POT_API int pot_prepare_clouds(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m,
                       int32_t d, const float *a, const float *b, int32_t precision,
                       void *ws, size_t ws_bytes, void *stream);

/* ---- General costs h(z) = (1/p) sum_k |z_k|^p ---------------------------
 *
 * ProgOT holds for any strictly convex translation-invariant cost (Sec. 3);
 * the coupling experiments of Sec. 5.2 and the map appendix use this h with
 * p = 1.5.  Clouds prepared with pot_prepare_clouds_pcost run every call
 * below with that cost instead of |x - y|^2:
 *   pot_sinkhorn_solve, pot_progot_solve: Alg. 1 / Alg. 2 on C_ij =
 *     h(x_i - y_j), the potentials in the same convention (P_ij =
 *     exp((f_i + g_j - C_ij)/eps)); eps_mode 0 uses theta * mean_ij C_ij/20
 *     per step (App. C);
 *   pot_entropic_map, pot_progot_map: the step of Alg. 2 / Alg. 3 for h,
 *     Xout = Xq - alpha grad h*(sum_j p_j grad h(Xq - y_j)), p_j =
 *     softmax_j((g_j - h(Xq - y_j))/eps), with grad h(z)_k = sign(z_k)
 *     |z_k|^(p-1) and grad h*(w)_k = sign(w_k) |w_k|^(1/(p-1)) (eq. Tent;
 *     alpha = 1 gives T itself);
 *   pot_coupling_metrics, pot_marginal_check, pot_diag_metrics: C in FP64 by
 *     direct differences.
 * FP32 only (there is no inner-product form to put on MFMA).  The cost
 * matrix of the current source iterate is either kept in the workspace
 * (n x ldc floats, rebuilt when the iterate moves; each potential update
 * then reads it once) or formed on the fly in every update (d powers per
 * pair, VALU-bound; the workspace does not grow with n m).  flags:
 *   POT_PCOST_AUTO       keep it when it takes at most 16 GiB;
 *   POT_PCOST_ON_THE_FLY never keep it;
 *   POT_PCOST_KEEP       keep it (n * m <= 2^36, else POT_ERR_INVALID).
 * Alg. 4 takes these clouds too (pot_eps_schedule_pcost_bytes); the
 * Sinkhorn divergence has its own general-cost entry point below; the
 * serving form takes squared-Euclidean clouds only.
 *   1 < p <= 16; p == 1.5 takes a square-root path, other p a log/exp path.
 *   n * m <= 2^43. */
#define POT_PCOST_AUTO 0
#define POT_PCOST_ON_THE_FLY 1
#define POT_PCOST_KEEP 2
POT_API size_t pot_workspace_bytes_pcost(int64_t n, int64_t m, int32_t d, float p, int32_t flags);
POT_API int pot_prepare_clouds_pcost(pot_clouds *c, const float *X, int64_t n, const float *Y,
                                     int64_t m, int32_t d, const float *a, const float *b, float p,
                                     int32_t flags, void *ws, size_t ws_bytes, void *stream);

typedef struct {
    int32_t iters;         /* full (f, g) iterations of the returned iterate     */
    int32_t converged;     /* 1 if err <= tau                                    */
    float err;             /* |P 1 - a|_1 of the returned (f, g)                 */
    double seconds;        /* host wall time of the call                         */
} pot_sinkhorn_info;

/* Alg. 1 Sink(a, X^(k), b, Y, eps, tau, f_init, g_init) on the current source
 * iterate c->xk.  Each iteration runs the f-update then the g-update (fused
 * cost + streaming log-sum-exp kernels, the n x m cost is never stored); the
 * row-marginal error of iteration t comes free from the f-update of t + 1.
 *   eps > 0; tau >= 0.  tau == 0 selects fixed-iteration mode: exactly
 *   max_iter iterations, status POT_OK.  max_iter >= 1.
 *   f_init (device, n) may be NULL: it cannot change the iterates because the
 *   first f-update overwrites f; g_init (device, m) NULL means zero.
 *   f (device, n) and g (device, m) receive the result; they may alias the
 *   init buffers.
 * Returns POT_WARN_NOT_CONVERGED when max_iter is hit with err > tau. */
POT_API int pot_sinkhorn_solve(pot_clouds *c, float eps, float tau, int32_t max_iter,
                       const float *f_init, const float *g_init, float *f, float *g,
                       pot_sinkhorn_info *info, void *stream);

/* The entropic map of eq. Tent against the target cloud of c with potential
 * g (device, m) at eps, followed by the McCann-type step:
 *   Xout_i = (1 - alpha) Xq_i + alpha sum_j softmax_j((g_j - |Xq_i - y_j|^2)/eps) y_j
 * Xq (device, nq*d) are arbitrary query points; Xout (device, nq*d) may alias
 * Xq.  0 <= alpha <= 1.  nq == 0 is a no-op. */
POT_API int pot_entropic_map(const pot_clouds *c, const float *g, float eps, const float *Xq,
                     int64_t nq, float alpha, float *Xout, void *stream);

typedef struct {
    int32_t K;             /* number of Sinkhorn solves, 1..POT_MAX_K            */
    int32_t alpha_sched;   /* 0 constant speed, 1 decelerated, 2 accelerated    */
    int32_t eps_mode;      /* 0: eps_k = theta * meancost(X^(k), Y)/20 (App. C);
                              1: eps_k = eps_explicit[k] (e.g. Alg. 4 output)   */
    float theta;
    const double *eps_explicit;  /* host, K values, eps_mode == 1 only          */
    float tau_first, tau_last;   /* tau_k linear from first to last (Sec. 4)    */
    int32_t max_iter;            /* per solve                                   */
    int32_t warm_start;          /* 0: (1 - alpha_k) as in Alg. 2; 1: (1 - alpha_{k-1}) */
} pot_progot_params;

typedef struct {
    int32_t K;
    int32_t iters[POT_MAX_K];    /* Sinkhorn iterations of each solve           */
    int32_t converged;           /* 1 if every solve met its tau                */
    float eps[POT_MAX_K], alpha[POT_MAX_K], err[POT_MAX_K];
    double seconds;
} pot_progot_info;

/* Alg. 2 ProgOT(a, X, b, Y, (eps_k, alpha_k, tau_k)_k).  Resets c->xk to X,
 * then for k = 0..K-1: eps_k, warm start, Sinkhorn to tau_k, store g^(k) in
 * G[k], and (k < K-1) move c->xk in place along the McCann-type step.  On
 * return c->xk holds X^(K-1), the source of the returned coupling
 * P = exp((f (+) g^(K-1) - C(X^(K-1), Y))/eps_{K-1}); c->mean_cost matches it.
 *   f (device, n): the last solve's f.  G (device, K*m): g^(0..K-1).
 *   TX (device, n*d) or NULL: X^(K) = T_{K-1}(X^(K-1)) (alpha_{K-1} = 1).
 * The fitted map of Alg. 3 is (Y, G, info->eps, info->alpha). */
POT_API int pot_progot_solve(pot_clouds *c, const pot_progot_params *p, float *f, float *G,
                     float *TX, pot_progot_info *info, void *stream);

/* Alg. 3 T_Prog[b, Y, (g^(k), eps_k, alpha_k)_k] at nq query points: y <- x,
 * then y <- (1 - alpha_k) y + alpha_k T_k(y) for k = 0..K-1 with alpha_{K-1}
 * reset to 1.  G (device, K*m); eps, alpha (host, K floats); Xq, Yout
 * (device, nq*d), may alias. */
POT_API int pot_progot_map(const pot_clouds *c, int32_t K, const float *G, const float *eps,
                   const float *alpha, const float *Xq, int64_t nq, float *Yout, void *stream);

/* Final check in FP64 on the current source iterate c->xk: with C_ij =
 * |x_i - y_j|^2 evaluated in FP64 by direct differences,
 *   out[0] = |P 1 - a|_1, out[1] = |P^T 1 - b|_1,
 *   out[2] = <f, a> + <g, b> - eps sum_ij P_ij   (the dual of eq. entdual),
 * the marginal criterion of the coupling experiments (Sec. 5.2).
 * f (device, n), g (device, m); out (host, 3 doubles).  Blocks. */
POT_API int pot_marginal_check(const pot_clouds *c, const float *f, const float *g, float eps,
                       double *out, void *stream);

/* Metrics of the coupling P = exp((f (+) g - C(c->xk, Y))/eps), one FP64
 * pass over all pairs (cost in FP64, cross term on FP64 MFMA):
 *   out[0] = |P 1 - a|_1, out[1] = |P^T 1 - b|_1,
 *   out[2] = <f, a> + <g, b> - eps sum_ij P_ij (the objective of eq.
 *            entdual, OT_eps of the Sinkhorn divergence, eq. sink_div),
 *   out[3] = <P, C> (transport cost), out[4] = sum_ij P_ij log P_ij,
 *   out[5] = sum_ij P_ij.
 * f (device, n), g (device, m); out (host, 6 doubles).  Blocks. */
POT_API int pot_coupling_metrics(const pot_clouds *c, const float *f, const float *g, float eps,
                                 double *out, void *stream);

/* Diagonal metrics of the coupling for n == m (the coupling-recovery
 * benchmark of Sec. 5.3, where the true coupling is the identity / n):
 *   out[0] = Tr P = sum_i P_ii,
 *   out[1] = KL(I/n || P) = -log n - (1/n) sum_i log P_ii,
 * with P_ii = exp((f_i + g_i - |x_i - y_i|^2)/eps) in FP64, O(n d).
 * POT_ERR_INVALID if n != m.  Blocks. */
POT_API int pot_diag_metrics(const pot_clouds *c, const float *f, const float *g, float eps,
                             double *out, void *stream);

/* Sinkhorn divergence (eq. sink_div) between weighted clouds X (n x d) and
 * Y (m x d), device pointers, a/b device weights or NULL (uniform):
 *   D = OT_eps(X, Y) - (OT_eps(X, X) + OT_eps(Y, Y)) / 2,
 * OT_eps the objective of eq. entdual at Alg. 1's FP32 solution to tau,
 * <f, a> + <g, b> - eps (the returned iterate ends with a g-update, so the
 * coupling's mass is 1), with FP64 dot products.  eps = 0 selects the
 * paper's eps_D = 5 % of the mean cost within Y.  out (host, 5 doubles): D,
 * OT(X,Y), OT(X,X), OT(Y,Y), eps.
 * ws (device): pot_sinkhorn_divergence_bytes(n, m, d) bytes, reused by the
 * three solves.  POT_WARN_NOT_CONVERGED if a solve hit max_iter.  Blocks. */
POT_API size_t pot_sinkhorn_divergence_bytes(int64_t n, int64_t m, int32_t d);
POT_API int pot_sinkhorn_divergence(const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                                    const float *a, const float *b, float eps, float tau,
                                    int32_t max_iter, double *out, void *ws, size_t ws_bytes,
                                    void *stream);
/* The same divergence with the cost h = (1/p)|.|_p^p (1 < p <= 16), as the
 * map appendix evaluates its 1.5-norm experiments: the three solves run on
 * general-cost clouds (see pot_prepare_clouds_pcost) and eps = 0 selects
 * 5 % of the mean of h within Y.  Workspace:
 * pot_sinkhorn_divergence_pcost_bytes(n, m, d, p) (0 if invalid). */
POT_API size_t pot_sinkhorn_divergence_pcost_bytes(int64_t n, int64_t m, int32_t d, float p);
POT_API int pot_sinkhorn_divergence_pcost(const float *X, int64_t n, const float *Y, int64_t m,
                                          int32_t d, const float *a, const float *b, float p,
                                          float eps, float tau, int32_t max_iter, double *out,
                                          void *ws, size_t ws_bytes, void *stream);

/* The same divergence for callers that cannot allocate memory (code under
 * HIP graph capture set-up, tight serving loops, harnesses that forbid
 * allocation): no workspace argument; the call calls no hipMalloc, hipFree,
 * hipHostMalloc or event creation.  Its workspace is a static device array of
 * POT_STATIC_SCRATCH_BYTES per GPU, part of the library's code object, held
 * from the first call on a device until the process ends; its device address
 * is looked up once per device (the device current at the call, which must
 * own `stream`).  Pairs whose pot_sinkhorn_divergence_bytes(n, m, d) exceeds
 * that size return POT_ERR_NOMEM before any work (e.g. n = m = 32768 at
 * d = 64 fit).  Every call on one GPU shares the array and leaves its
 * contents behind; each call writes every region before reading it, so
 * nothing needs clearing, but calls that overlap on one GPU (two host threads,
 * or two streams in flight) race and must be serialised by the caller.  The
 * error sums of the Sinkhorn loop are copied back and checked after every
 * iteration (one stream synchronisation each), so the call returns exactly
 * what pot_sinkhorn_divergence returns, a little more slowly for short
 * iterations.  Arguments, results and errors otherwise as above.  Blocks. */
#define POT_STATIC_SCRATCH_BYTES (32u << 20)
POT_API int pot_sinkhorn_divergence_noalloc(const float *X, int64_t n, const float *Y, int64_t m,
                                            int32_t d, const float *a, const float *b, float eps,
                                            float tau, int32_t max_iter, double *out, void *stream);

/* ---- Alg. 4 (eps-scheduler) ------------------------------------------------
 *
 * The schedule of regularisations that Alg. 2 consumes (pass the result as
 * pot_progot_params.eps_explicit with eps_mode = 1):
 *   eps_0 = c->mean_cost / 20 (the prepared pair: call before the source
 *           iterate moves, i.e. after pot_prepare_clouds),
 *   sigma = mean_lj |y_l - y_j|^2 / 20 (closed form from the targets),
 *   for each grid scale s_p: Sink(b, Y, b, Y, s_p sigma, tau) (Alg. 1), the
 *           one-step entropic map of the hold-out targets Y_test (alpha = 1)
 *           and err_p = sum |y~ - T_p(y~)|^2,
 *   p* = first argmin, eps_final = s_{p*} sigma,
 *   eps_k = (1 - t_k) beta0 eps_0 + t_k eps_final, t_k = 1 - prod_{l=1..k}
 *           (1 - alpha_l) of the alpha schedule (K = 1: eps_final).
 * The grid solves run in FP32 and advance together in grouped launches; each
 * gets the same result as pot_sinkhorn_solve on (Y, Y) at its eps.
 *   c: prepared clouds (any precision; only Y, b, m, d, mean_cost and the
 *      cost are used).
 *   Y_test (device, m_test*d): hold-out targets.
 *   s_grid (host, n_grid doubles > 0), 1 <= n_grid <= POT_MAX_GRID.
 *   eps_out (host, K doubles); err_out (host, n_grid doubles) and p_star
 *   (host) may be NULL.  ws (device): pot_eps_schedule_bytes() bytes.
 * Returns POT_WARN_NOT_CONVERGED (outputs valid) when a grid solve hit
 * max_iter.  Blocks. */
#define POT_MAX_GRID 64
POT_API size_t pot_eps_schedule_bytes(int64_t m, int64_t m_test, int32_t d, int32_t n_grid);
/* Clouds prepared with pot_prepare_clouds_pcost run Alg. 4 with their cost h
 * (eps_0 and sigma from the mean of h, grid solves and maps with h; the
 * hold-out score stays the squared distance).  The grid solves then run one
 * after another on the resident (Y, Y) cost matrix, in a workspace of
 * pot_eps_schedule_pcost_bytes(m, m_test, d, n_grid, p) bytes. */
POT_API size_t pot_eps_schedule_pcost_bytes(int64_t m, int64_t m_test, int32_t d, int32_t n_grid,
                                            float p);
POT_API int pot_eps_schedule(const pot_clouds *c, const float *Y_test, int64_t m_test, int32_t K,
                             int32_t alpha_sched, const double *s_grid, int32_t n_grid, float beta0,
                             float tau, int32_t max_iter, double *eps_out, double *err_out,
                             int32_t *p_star, void *ws, size_t ws_bytes, void *stream);

/* ---- Serving form: continuous batching of ProgOT solves ------------------
 *
 * A server advances many independent ProgOT solves (Alg. 2) of uneven sizes
 * together.  The caller gives it one device arena; each admitted request
 * takes a workspace of pot_server_request_bytes() from it (first fit), so
 * admission is by HBM footprint, bounded also by max_active slots.  Each
 * pot_server_step is one tick: up to 16 Sinkhorn iterations of every
 * active request, each sub-step with all f-updates in one grouped kernel
 * launch per padded dimension and likewise all g-updates (the stop rule runs
 * on the device), then one read-back of all their control words; a request
 * whose solve met its tau takes its McCann step and starts the next ProgOT
 * step at the following tick, and a request
 * submitted between ticks joins at the next one.  The grouped launches are
 * persistent kernels (a grid of the workgroups the chip holds at once, each
 * walking the tick's work list of (request, row tile, column split) items),
 * and the maps of every request whose solve ended in a tick (its McCann step
 * or its final map) run in one grouped map launch per padded dimension.  A
 * request computes exactly what pot_progot_solve computes for it alone (bit
 * for bit): same device bodies, same column splits, same host arithmetic.
 * FP32 cross term, uniform weights.  Calls on one server are not
 * thread-safe. */
typedef struct pot_server pot_server;

#define POT_SERVER_MAX_ACTIVE 1024

/* Device bytes the server keeps for itself at the start of the arena. */
POT_API size_t pot_server_arena_overhead(int32_t max_active);
/* Device bytes one request of these sizes occupies in the arena (0 if invalid). */
POT_API size_t pot_server_request_bytes(int64_t n, int64_t m, int32_t d);

/* arena (device, arena_bytes) is owned by the caller and must outlive the
 * server; stream is the hipStream_t every launch goes to (as void*).
 * 1 <= max_active <= POT_SERVER_MAX_ACTIVE. */
POT_API int pot_server_create(pot_server **out, void *arena, size_t arena_bytes,
                              int32_t max_active, void *stream);

/* Admit one solve: X (device, n*d), Y (device, m*d), parameters as for
 * pot_progot_solve; outputs f (device, n), G (device, K*m), TX (device, n*d,
 * or NULL) are written when the request finishes.  Inputs and outputs must
 * stay valid until then.  Returns POT_BUSY when no slot or no arena space is
 * free now (retry after a step), POT_ERR_NOMEM when the request can never fit
 * the arena.  The prepare kernels are enqueued at once. */
POT_API int pot_server_submit(pot_server *srv, const float *X, int64_t n, const float *Y,
                              int64_t m, int32_t d, const pot_progot_params *p, float *f,
                              float *G, float *TX, int64_t *rid);

/* One tick (blocks on the stream).  n_active: requests still in flight;
 * n_finished: requests that finished in this tick (their outputs are in
 * place).  A request that fails (a non-finite mean cost or marginal error,
 * e.g. from a NaN in its clouds) finishes with its status, which
 * pot_server_poll reports; the tick itself still returns POT_OK and the other
 * requests are unaffected.  POT_ERR_DEVICE when a HIP call fails. */
POT_API int pot_server_step(pot_server *srv, int32_t *n_active, int32_t *n_finished);

/* POT_BUSY while request rid is in flight; once finished, fills info (may be
 * NULL), forgets the request and returns its status (POT_OK,
 * POT_WARN_NOT_CONVERGED or an error).  POT_ERR_INVALID for an unknown rid. */
POT_API int pot_server_poll(pot_server *srv, int64_t rid, pot_progot_info *info);

/* Waits for the stream and frees the server's host state (not the arena). */
POT_API int pot_server_destroy(pot_server *srv);

/* Kernel timing, a tracing aid.  While enabled (process-wide), launches of
 * the potential-update kernel (the f- and g-update) and of the entropic-map
 * kernel are bracketed by HIP timing events, recorded by the dispatch itself
 * on the stream it is launched on.  pot_timing_enable(every), every >= 1,
 * clears the counters and times launches 0, every, 2 every, ... of each of
 * the two kernels (1: every launch; a larger stride samples, which keeps the
 * cost of the events -- two per timed launch, and the host work to record
 * them -- off short kernels); pot_timing_enable(0) stops; every < 0 is
 * POT_ERR_INVALID.  pot_timing_read waits for the recorded events and
 * returns the summed milliseconds and counts of the timed launches (any
 * pointer may be NULL).  Calls are serialised by a mutex. */
POT_API int pot_timing_enable(int every);
POT_API int pot_timing_read(double *lse_ms, int64_t *lse_launches, double *map_ms,
                            int64_t *map_launches);

/* Message for a pot_status code (static string). */
POT_API const char *pot_status_string(int code);

/* Library version, "major.minor.patch". */
POT_API const char *pot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PROGOT_H */
