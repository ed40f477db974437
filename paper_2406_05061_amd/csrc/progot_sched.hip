// Alg. 4 (the eps-scheduler) on the GPU.  (For the general cost
// h = (1/p)|.|_p^p, see schedule_pcost below.)
//
// eps_0 is the mean cost of the caller's pair / 20 and sigma the mean cost of
// the targets with themselves / 20 (closed form from the targets' FP64
// moments).  For every scale s_p of the grid, Alg. 1 is run on (b, Y, b, Y)
// at eps_p = s_p sigma to tolerance tau; all grid points advance together,
// one grouped f-update launch and one grouped g-update launch per iteration
// (the same kernels and bodies as a solve on its own, so each grid point
// gets the bits pot_sinkhorn_solve would give it), with the stop rule of
// Alg. 1 checked per grid point on the host exactly as in a single solve.
// The hold-out targets are then mapped by the one-step entropic map
// (alpha = 1) of each solve and scored by err_p = sum |y~ - T_p(y~)|^2 (FP64
// sum).  With p* the first argmin, eps_final = s_{p*} sigma and the schedule
// is eps_k = (1 - t_k) beta0 eps_0 + t_k eps_final, t_k = 1 - prod_{l=1..k}
// (1 - alpha_l) (K = 1: eps_final).

#include "progot.h"
#include "progot_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

using namespace pot::host;
using pot::LseJob;

namespace {

constexpr int kSqBlocks = 256;

// Per-block FP64 partial sums of (a_i - b_i)^2 over len floats.
__global__ __launch_bounds__(256) void sqdist_partial(const float *__restrict__ A,
                                                      const float *__restrict__ B, int64_t len,
                                                      double *__restrict__ part) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < len; i += (int64_t)gridDim.x * 256) {
        const double e = (double)A[i] - (double)B[i];
        s = fma(e, e, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// Workspace: the (Y, Y) pair, then one block of buffers per grid point
// (ping-pong potentials, split partials, error partials), the job tables,
// the error sums, the mapped hold-out targets and the FP64 partials.
struct SchedLayout {
    Layout cy;
    size_t f0, f1, g0, g1, pm, ps, errp, per_p;  // within one grid point's block
    size_t grid, jobs, ctl, ty, sq, total;
};

// Sinkhorn iterations enqueued per host read-back of the stop words: the
// first blocks are short (large-eps grid points stop within a few
// iterations), later ones up to kMaxBlockIters.
constexpr int kFirstBlockIters = 4;
constexpr int kMaxBlockIters = 32;

SchedLayout sched_plan(int64_t m, int64_t mt, int32_t d, int32_t G) {
    SchedLayout S{};
    S.cy = plan(m, m, d, POT_PREC_FP32);
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = a256(o + bytes); return r; };
    S.f0 = take((size_t)m * 4);
    S.f1 = take((size_t)m * 4);
    S.g0 = take((size_t)m * 4);
    S.g1 = take((size_t)m * 4);
    S.pm = take((size_t)pot::kMaxSplit * m * 4);
    S.ps = take((size_t)pot::kMaxSplit * m * 4);
    S.errp = take((((size_t)m + 255) / 256) * 4);
    S.per_p = o;
    S.grid = a256(S.cy.total);
    size_t off = S.grid + (size_t)G * S.per_p;
    auto take2 = [&](size_t bytes) { size_t r = off; off = a256(off + bytes); return r; };
    S.jobs = take2(sizeof(LseJob) * 2 * (size_t)G * kMaxBlockIters);
    S.ctl = take2(sizeof(int) * 2 * (size_t)G);
    S.ty = take2((size_t)mt * d * 4);
    S.sq = take2(kSqBlocks * sizeof(double) * (size_t)G);
    S.total = off;
    return S;
}

struct GridPoint {
    float eps;
    float *fb[2], *gb[2];
    float *pm, *ps, *errp;
    bool done = false, converged = false;
    int iters = 0;
    float err = 0.f;
    const float *g = nullptr;
};

LseJob point_job(const LseJob &base, const GridPoint &q) {
    LseJob j = base;
    j.eps = q.eps;
    j.part_m = q.pm;
    j.part_s = q.ps;
    return j;
}

// General costs: the (Y, Y) pair as general-cost clouds, then the mapped
// hold-out targets and the FP64 partials.
struct PSchedLayout {
    Layout cy;
    size_t ty, sq, total;
};

PSchedLayout psched_plan(int64_t m, int64_t mt, int32_t d, float p) {
    PSchedLayout S{};
    S.cy = plan(m, m, d, POT_PREC_FP32, p, pcost_keep(m, m, POT_PCOST_AUTO) == 1);
    size_t off = a256(S.cy.total);
    S.ty = off;
    off = a256(off + (size_t)mt * d * 4);
    S.sq = off;
    S.total = a256(off + kSqBlocks * sizeof(double));
    return S;
}

bool valid_pcost_pair(int64_t m, int32_t d, float p) {
    return p != 0.f && valid_cost_p(p) && valid_sizes(m, m, d, POT_PREC_FP32) &&
           pot::pcost_matrix_blocks(m, m) <= 0x7fffffff;
}

// Hold-out score err_p = sum |y~ - T_p(y~)|^2 of one grid solve: the map of
// the hold-out targets into ty and the FP64 partials of the squared distance
// into sq_dev (kSqBlocks doubles), enqueued only.
int enqueue_holdout(const pot_clouds *cy, const float *g, float eps, const float *Y_test, int64_t mt,
                    float *ty, double *sq_dev, hipStream_t s) {
    int st = run_map(cy, g, eps, Y_test, mt, 1.f, ty, s);
    if (st != POT_OK) return st;
    hipLaunchKernelGGL(sqdist_partial, dim3(kSqBlocks), dim3(256), 0, s, Y_test, ty,
                       mt * (int64_t)cy->d, sq_dev);
    POT_TRY(hipGetLastError());
    return POT_OK;
}

// Sum of the partials read back (in order, so the score does not depend on
// how many grid points were scored together).
int finish_holdout(const double *sq, double *score) {
    double tot = 0.0;
    for (int i = 0; i < kSqBlocks; ++i) tot += sq[i];
    if (!std::isfinite(tot)) return POT_ERR_NUMERIC;
    *score = tot;
    return POT_OK;
}

int holdout_score(const pot_clouds *cy, const float *g, float eps, const float *Y_test, int64_t mt,
                  float *ty, double *sq_dev, double *score, hipStream_t s) {
    int st = enqueue_holdout(cy, g, eps, Y_test, mt, ty, sq_dev, s);
    if (st != POT_OK) return st;
    std::vector<double> sq(kSqBlocks);
    POT_TRY(hipMemcpyAsync(sq.data(), sq_dev, sizeof(double) * kSqBlocks, hipMemcpyDeviceToHost, s));
    POT_TRY(hipStreamSynchronize(s));
    return finish_holdout(sq.data(), score);
}

// eps_k from the selected scale (the last lines of Alg. 4).
void write_schedule(int K, int alpha_sched, double beta0, double eps0, double eps_final,
                    double *eps_out) {
    float alpha[POT_MAX_K];
    alpha_schedule(K, alpha_sched, alpha);
    if (K == 1) {
        eps_out[0] = eps_final;
        return;
    }
    double prod = 1.0;
    for (int k = 0; k < K; ++k) {
        if (k > 0) prod *= 1.0 - (double)alpha[k];
        const double tk = 1.0 - prod;
        eps_out[k] = (1.0 - tk) * beta0 * eps0 + tk * eps_final;
    }
}

// Alg. 4 for the cost h = (1/p)|.|_p^p: sigma from the mean of h within Y
// (the (Y, Y) cost matrix), and the grid solves one after another on that
// resident matrix with the single-problem loop; the hold-out score is the
// same squared distance as for the squared-Euclidean cost.
int schedule_pcost(const pot_clouds *c, const float *Y_test, int64_t mt, int32_t K,
                   int32_t alpha_sched, const double *s_grid, int32_t n_grid, float beta0,
                   float tau, int32_t max_iter, double *eps_out, double *err_out, int32_t *p_star,
                   void *ws, size_t ws_bytes, hipStream_t s) {
    const int64_t m = c->m;
    const int d = c->d;
    if (!valid_pcost_pair(m, d, c->cost_p)) return POT_ERR_INVALID;
    const PSchedLayout S = psched_plan(m, mt, d, c->cost_p);
    if (ws_bytes < S.total) return POT_ERR_NOMEM;
    char *base = static_cast<char *>(ws);
    pot_clouds cy;
    bind_clouds(&cy, c->Y, m, c->Y, m, d, c->b, c->b, POT_PREC_FP32, ws, S.cy.total, S.cy, c->cost_p,
                pcost_keep(m, m, POT_PCOST_AUTO) == 1);
    std::vector<double> mom(moments_len(d));
    int st = enqueue_prepare(&cy, S.cy, mom.data(), s);
    if (st != POT_OK) return st;
    POT_TRY(hipStreamSynchronize(s));
    if ((st = finish_moments(&cy, mom.data())) != POT_OK) return st;
    if ((st = refresh_pcost(&cy, S.cy, s)) != POT_OK) return st;
    const double sigma = cy.mean_cost / 20.0;
    const double eps0 = c->mean_cost / 20.0;
    if (!(sigma > 0.0) || !(eps0 > 0.0)) return POT_ERR_NUMERIC;
    float *ty = reinterpret_cast<float *>(base + S.ty);
    double *sq_dev = reinterpret_cast<double *>(base + S.sq);
    std::vector<double> score(n_grid);
    bool all = true;
    for (int q = 0; q < n_grid; ++q) {
        const float eps = (float)(s_grid[q] * sigma);
        if (!finite_pos(eps)) return POT_ERR_INVALID;
        SinkOut r;
        if ((st = run_sinkhorn(&cy, S.cy, eps, tau, max_iter, nullptr, 1.f, &r, s)) != POT_OK) return st;
        all = all && r.converged;
        if ((st = holdout_score(&cy, r.g, eps, Y_test, mt, ty, sq_dev, &score[q], s)) != POT_OK)
            return st;
    }
    int best = 0;
    for (int q = 1; q < n_grid; ++q)
        if (score[q] < score[best]) best = q;
    write_schedule(K, alpha_sched, beta0, eps0, s_grid[best] * sigma, eps_out);
    if (err_out)
        for (int q = 0; q < n_grid; ++q) err_out[q] = score[q];
    if (p_star) *p_star = best;
    return all ? POT_OK : POT_WARN_NOT_CONVERGED;
}

}  // namespace

extern "C" {

size_t pot_eps_schedule_pcost_bytes(int64_t m, int64_t m_test, int32_t d, int32_t n_grid, float p) {
    if (!valid_pcost_pair(m, d, p) || m_test < 1 || n_grid < 1 || n_grid > POT_MAX_GRID) return 0;
    return psched_plan(m, m_test, d, p).total;
}

size_t pot_eps_schedule_bytes(int64_t m, int64_t m_test, int32_t d, int32_t n_grid) {
    if (!valid_sizes(m, m, d, POT_PREC_FP32) || m_test < 1 || n_grid < 1 || n_grid > POT_MAX_GRID)
        return 0;
    return sched_plan(m, m_test, d, n_grid).total;
}

int pot_eps_schedule(const pot_clouds *c, const float *Y_test, int64_t m_test, int32_t K,
                     int32_t alpha_sched, const double *s_grid, int32_t n_grid, float beta0,
                     float tau, int32_t max_iter, double *eps_out, double *err_out,
                     int32_t *p_star, void *ws, size_t ws_bytes, void *stream) {
    if (!valid_clouds(c) || !Y_test || m_test < 1 || K < 1 || K > POT_MAX_K || alpha_sched < 0 ||
        alpha_sched > 2 || !s_grid || n_grid < 1 || n_grid > POT_MAX_GRID || !finite_pos(beta0) ||
        !finite_pos(tau) || max_iter < 1 || !eps_out || !ws)
        return POT_ERR_INVALID;
    for (int p = 0; p < n_grid; ++p)
        if (!(std::isfinite(s_grid[p]) && s_grid[p] > 0.0)) return POT_ERR_INVALID;
    if (c->cost_p != 0.f)
        return schedule_pcost(c, Y_test, m_test, K, alpha_sched, s_grid, n_grid, beta0, tau, max_iter,
                              eps_out, err_out, p_star, ws, ws_bytes, static_cast<hipStream_t>(stream));
    const int64_t m = c->m;
    const int d = c->d;
    const SchedLayout S = sched_plan(m, m_test, d, n_grid);
    if (ws_bytes < S.total) return POT_ERR_NOMEM;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(ws);

    // the (Y, Y) pair with the target weights on both sides; sigma from its
    // mean cost (closed form from the FP64 moments)
    pot_clouds cy;
    bind_clouds(&cy, c->Y, m, c->Y, m, d, c->b, c->b, POT_PREC_FP32, ws, S.cy.total, S.cy);
    std::vector<double> mom(moments_len(d));
    int st = enqueue_prepare(&cy, S.cy, mom.data(), s);
    if (st != POT_OK) return st;
    POT_TRY(hipStreamSynchronize(s));
    if ((st = finish_moments(&cy, mom.data())) != POT_OK) return st;
    const double sigma = cy.mean_cost / 20.0;
    const double eps0 = c->mean_cost / 20.0;
    if (!(sigma > 0.0) || !(eps0 > 0.0)) return POT_ERR_NUMERIC;

    std::vector<GridPoint> pts(n_grid);
    for (int p = 0; p < n_grid; ++p) {
        char *blk = base + S.grid + (size_t)p * S.per_p;
        GridPoint &q = pts[p];
        q.eps = (float)(s_grid[p] * sigma);
        if (!finite_pos(q.eps)) return POT_ERR_INVALID;
        q.fb[0] = reinterpret_cast<float *>(blk + S.f0);
        q.fb[1] = reinterpret_cast<float *>(blk + S.f1);
        q.gb[0] = reinterpret_cast<float *>(blk + S.g0);
        q.gb[1] = reinterpret_cast<float *>(blk + S.g1);
        q.pm = reinterpret_cast<float *>(blk + S.pm);
        q.ps = reinterpret_cast<float *>(blk + S.ps);
        q.errp = reinterpret_cast<float *>(blk + S.errp);
    }
    LseJob *jobs_dev = reinterpret_cast<LseJob *>(base + S.jobs);
    int *ctl_dev = reinterpret_cast<int *>(base + S.ctl);
    const LseJob fbase = f_job(&cy, S.cy, 1.f), gbase = g_job(&cy, S.cy, 1.f);

    // Alg. 1 for every grid point, advanced together.  Iteration t: f_t
    // (whose error partials are the row-marginal error of iterate t-1), then
    // g_t; at t = max_iter + 1 only the f-update, for the error of the last
    // iterate.  The stop rule runs on the device: the error sum of f_t sets
    // the grid point's control word {stop iterate, error bits} once the error
    // of iterate t-1 meets tau (or t-1 = max_iter), and every later update of
    // that grid point is skipped, so its iterate t-1 stays intact in the
    // ping-pong buffers (f_t writes the other one).  Blocks of iterations are
    // enqueued between read-backs of the control words; each block's job
    // tables go up in one copy.
    POT_TRY(hipMemsetAsync(ctl_dev, 0, sizeof(int) * 2 * (size_t)n_grid, s));
    std::vector<LseJob> tab((size_t)2 * n_grid * kMaxBlockIters);
    std::vector<pot::GroupPlan> plans(2 * kMaxBlockIters);
    std::vector<int> act, ctl(2 * (size_t)n_grid);
    int t0 = 1, block = kFirstBlockIters;
    while (true) {
        act.clear();
        for (int p = 0; p < n_grid; ++p)
            if (!pts[p].done) act.push_back(p);
        if (act.empty()) break;
        if (t0 > max_iter + 1) return POT_ERR_DEVICE;   // every grid point stops by then
        const int na = (int)act.size();
        const int nt = std::min<int64_t>(block, (int64_t)max_iter + 1 - t0 + 1);
        for (int u = 0; u < nt; ++u) {
            const int t = t0 + u;
            LseJob *fj = tab.data() + (size_t)2 * na * u, *gj = fj + na;
            for (int k = 0; k < na; ++k) {
                const int p = act[k];
                const GridPoint &q = pts[p];
                LseJob f = point_job(fbase, q);
                f.vpot = t == 1 ? nullptr : q.gb[(t - 1) & 1];
                f.pot_old = t == 1 ? nullptr : q.fb[(t - 1) & 1];
                f.pot_out = q.fb[t & 1];
                f.err_part = q.errp;
                f.ctl = ctl_dev + 2 * p;
                f.iter = t - 1;
                f.max_iter = max_iter;
                f.tau = tau;
                fj[k] = f;
                LseJob g = point_job(gbase, q);
                g.vpot = q.fb[t & 1];
                g.pot_out = q.gb[t & 1];
                g.err_part = nullptr;
                g.ctl = f.ctl;
                gj[k] = g;
            }
            POT_TRY(pot::plan_lse_update_group(fj, na, &plans[2 * u]));
            POT_TRY(pot::plan_lse_update_group(gj, na, &plans[2 * u + 1]));
        }
        POT_TRY(hipMemcpyAsync(jobs_dev, tab.data(), sizeof(LseJob) * 2 * na * nt, hipMemcpyHostToDevice, s));
        for (int u = 0; u < nt; ++u) {
            const int t = t0 + u;
            const LseJob *fd = jobs_dev + (size_t)2 * na * u;
            POT_TRY(pot::enqueue_lse_update_group(fd, na, plans[2 * u], nullptr, s));
            if (t <= max_iter) POT_TRY(pot::enqueue_lse_update_group(fd + na, na, plans[2 * u + 1], nullptr, s));
        }
        POT_TRY(hipMemcpyAsync(ctl.data(), ctl_dev, sizeof(int) * 2 * n_grid, hipMemcpyDeviceToHost, s));
        // the host tables above stay untouched until the stream has read them
        POT_TRY(hipStreamSynchronize(s));
        for (int p : act) {
            GridPoint &q = pts[p];
            const int it = ctl[2 * p];
            if (it == 0) continue;
            float err;
            std::memcpy(&err, &ctl[2 * p + 1], sizeof(float));
            if (!std::isfinite(err)) return POT_ERR_NUMERIC;
            q.done = true;
            q.converged = err <= tau;
            q.iters = it;
            q.err = err;
            q.g = q.gb[it & 1];
        }
        t0 += nt;
        block = std::min(2 * block, kMaxBlockIters);
    }

    // hold-out scores: every grid point's map and partials, one read-back
    float *ty = reinterpret_cast<float *>(base + S.ty);
    double *sq_dev = reinterpret_cast<double *>(base + S.sq);
    for (int p = 0; p < n_grid; ++p)
        if ((st = enqueue_holdout(&cy, pts[p].g, pts[p].eps, Y_test, m_test, ty,
                                  sq_dev + (size_t)p * kSqBlocks, s)) != POT_OK)
            return st;
    std::vector<double> sq((size_t)n_grid * kSqBlocks), score(n_grid);
    POT_TRY(hipMemcpyAsync(sq.data(), sq_dev, sizeof(double) * sq.size(), hipMemcpyDeviceToHost, s));
    POT_TRY(hipStreamSynchronize(s));
    for (int p = 0; p < n_grid; ++p)
        if ((st = finish_holdout(sq.data() + (size_t)p * kSqBlocks, &score[p])) != POT_OK) return st;
    int best = 0;
    for (int p = 1; p < n_grid; ++p)
        if (score[p] < score[best]) best = p;
    write_schedule(K, alpha_sched, beta0, eps0, s_grid[best] * sigma, eps_out);
    if (err_out)
        for (int p = 0; p < n_grid; ++p) err_out[p] = score[p];
    if (p_star) *p_star = best;
    bool all = true;
    for (const GridPoint &q : pts) all = all && q.converged;
    return all ? POT_OK : POT_WARN_NOT_CONVERGED;
}

}  // extern "C"
