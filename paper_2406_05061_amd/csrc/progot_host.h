// Host-side building blocks shared by the single-problem entry points and the
// serving scheduler, so both take exactly the same steps (same kernels, same
// splits, same host arithmetic) and a problem gets the same bits either way.
#pragma once

#include "progot.h"
#include "progot_internal.h"

#include <cstddef>
#include <cstdint>

namespace pot {
namespace host {

// Workspace regions of one pair of clouds (byte offsets, 256-byte aligned).
struct Layout {
    size_t xk, xsq, ysq, la, lb, xlp, ylp, ytl, f0, f1, g0, g1, pm, ps, errp, xst, yst, chr, chc,
        n64;
    size_t f2, g2;         // third potential slots of the single-problem Sinkhorn loop
    size_t yts;            // plain BF16 form: max |y| and the unscale of the FP16 copy
    size_t eslot;          // device slots of the error sums when they are copied back
                           // (entry points that allocate no pinned host memory)
    size_t cm, cmp, mpa;   // general costs: cost matrix, its block sums, map partials
    size_t total;
};

// cost_p = 0: squared-Euclidean cost; cost_p > 1: (1/p)|.|_p^p (FP32),
// keeping its n x m matrix in the workspace when keep_cost is set.
Layout plan(int64_t n, int64_t m, int32_t d, int32_t precision, float cost_p = 0.f,
            bool keep_cost = true);
bool valid_cost_p(float p);
// General costs: keep the cost matrix (flags 2), never (flags 1), or when
// it takes at most 16 GiB (flags 0).  Returns -1 for invalid flags.
int pcost_keep(int64_t n, int64_t m, int32_t flags);
// plan() of prepared clouds (their cost and whether they keep its matrix).
Layout plan_of(const pot_clouds *c);

template <typename T> T *at(const pot_clouds *c, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(c->ws) + off);
}

bool valid_sizes(int64_t n, int64_t m, int32_t d, int32_t precision);
bool valid_clouds(const pot_clouds *c);
bool finite_pos(float v);
double now_s();

// Fill the views of c over the workspace (no device work).
void bind_clouds(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                 const float *a, const float *b, int32_t precision, void *ws, size_t ws_bytes,
                 const Layout &L, float cost_p = 0.f, bool keep_cost = true);
// General costs: rebuild the cost matrix of the current source iterate (if
// kept) and set c->mean_cost from its sum (blocks until the sum is on the
// host).
int refresh_pcost(pot_clouds *c, const Layout &L, hipStream_t s);

// Number of doubles of a moments read-back: (sum_i x_i, sum |x|^2) for the
// source iterate and for the targets.
inline int moments_len(int d) { return 2 * (d + 1); }

// Enqueue xk = X, log weights, the targets' norms/copies/moments and the
// source's, then the moments' copy into `host` (2 (d+1) doubles, pinned or
// not: the caller synchronises before finish_moments).
int enqueue_prepare(pot_clouds *c, const Layout &L, double *host, hipStream_t s);
// Enqueue the source iterate's norms (unless norms_ready), BF16 copies and
// moments, and the copy.
int enqueue_moments(pot_clouds *c, const Layout &L, double *host, hipStream_t s,
                    bool norms_ready = false);
// True when the McCann step's map writes the moved source's squared norms
// itself (the FP32 squared-Euclidean form): then the moments pass after it
// skips the norm kernel.  The single-problem loop and the server both
// follow this, so a problem gets the same bits either way.
bool map_writes_norms(const pot_clouds *c);
// mean_ij |x_i - y_j|^2 = (1/n) sum |x|^2 + (1/m) sum |y|^2 - 2 xbar . ybar.
int finish_moments(pot_clouds *c, const double *host);

LseJob f_job(const pot_clouds *c, const Layout &L, float eps);
LseJob g_job(const pot_clouds *c, const Layout &L, float eps);

// alpha_k for k = 0..K-1 (0 constant speed, 1 decelerated, 2 accelerated).
void alpha_schedule(int K, int kind, float *alpha);
// eps_k, tau_k and the warm-start factor of step k of a ProgOT solve.
int step_values(const pot_progot_params *p, const float *alpha, int k, double mean_cost,
                float *eps, float *tau, float *gamma);
bool valid_params(const pot_progot_params *p);

// out_sqn (FP32 squared-Euclidean form only, else ignored): |Xout_i|^2.
int run_map(const pot_clouds *c, const float *g, float eps, const float *Xq, int64_t nq,
            float alpha, float *Xout, hipStream_t s, float *out_sqn = nullptr);

// Alg. 1 on c->xk as pot_sinkhorn_solve runs it; f and g point into the
// clouds' workspace and stay valid until the next solve on it.
struct SinkOut {
    int iters;
    float err;
    bool converged;
    const float *f, *g;
};
int run_sinkhorn(const pot_clouds *c, const Layout &L, float eps, float tau, int max_iter,
                 const float *g_init, float gamma, SinkOut *out, hipStream_t s);

}  // namespace host
}  // namespace pot

#define POT_TRY(expr)                                         \
    do {                                                      \
        hipError_t _e = (expr);                               \
        if (_e != hipSuccess) return POT_ERR_DEVICE;          \
    } while (0)
