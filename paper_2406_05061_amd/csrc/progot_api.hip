// C ABI and host driver of the progressive entropic OT hot path (gfx950).
//
// The host code owns no device memory: every buffer is a view into the caller's
// workspace, laid out by plan() from (n, m, d, precision).  Host-side state is
// limited to a small per-thread pinned buffer for scalar read-backs (with the
// event that marks the end of the last solve's work on it).

#include "progot.h"
#include "progot_host.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

namespace pot {
namespace host {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

Layout plan(int64_t n, int64_t m, int32_t d, int32_t precision, float cost_p, bool keep_cost) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t nm = (size_t)std::max(n, m);
    L.xk = take((size_t)n * d * 4);
    L.xsq = take((size_t)n * 4);
    L.ysq = take((size_t)m * 4);
    L.la = take((size_t)n * 4);
    L.lb = take((size_t)m * 4);
    // BF16 forms: [hi | lo] row copies padded to bf16_dim(d), and the
    // transposed target copy used by the projection product.
    const bool lp = precision != POT_PREC_FP32;
    const size_t Dp = (size_t)pot::bf16_dim(d);
    L.xlp = take(lp ? 2 * (size_t)pot::bf16_mpad(n) * Dp * 2 : 0);
    L.ylp = take(lp ? 2 * (size_t)pot::bf16_mpad(m) * Dp * 2 : 0);
    L.ytl = take(lp ? 2 * Dp * (size_t)pot::bf16_mpad(m) * 2 : 0);
    L.yts = take(precision == POT_PREC_BF16 ? 2 * sizeof(float) : 0);
    L.f0 = take((size_t)n * 4);
    L.f1 = take((size_t)n * 4);
    L.g0 = take((size_t)m * 4);
    L.g1 = take((size_t)m * 4);
    L.f2 = take((size_t)n * 4);
    L.g2 = take((size_t)m * 4);
    L.pm = take((size_t)pot::kMaxSplit * nm * 4);
    L.ps = take((size_t)pot::kMaxSplit * nm * 4);
    // error partials: one per 256 rows from the merge kernel, or one per 4
    // rows from the fused row update of the general-cost path
    L.errp = take((cost_p != 0.f ? (nm + 3) / 4 : (nm + 255) / 256) * 4);
    L.xst = take((size_t)pot::cloud_stat_blocks(n) * (d + 1) * 8);
    L.yst = take((size_t)pot::cloud_stat_blocks(m) * (d + 1) * 8);
    L.chr = take((size_t)pot::fp64_check_blocks(n) * pot::kCheckParts * 8);
    L.chc = take((size_t)pot::fp64_check_blocks(m) * pot::kCheckParts * 8);
    L.n64 = take(std::max<size_t>((size_t)n + (size_t)m, 512) * 8);   // FP64 norms / partials
    L.eslot = take(4 * sizeof(float));
    // general costs: the cost matrix of (xk, Y), its block sums (+ the
    // total), and the accumulator partials of the split map kernel
    const bool pc = cost_p != 0.f;
    L.cm = take(pc && keep_cost ? (size_t)n * (size_t)pot::pcost_ldc(m) * 4 : 0);
    L.cmp = take(pc ? ((size_t)pot::pcost_matrix_blocks(n, m) + 1) * 8 : 0);
    L.mpa = take(pc ? (size_t)pot::pcost_map_max_split() * n * pot::pcost_pad_dim(d) * 4 : 0);
    L.total = off;
    return L;
}

bool valid_cost_p(float p) { return p == 0.f || (std::isfinite(p) && p > 1.f && p <= 16.f); }

int pcost_keep(int64_t n, int64_t m, int32_t flags) {
    const double entries = (double)n * (double)pot::pcost_ldc(m);
    switch (flags) {
        case POT_PCOST_AUTO: return entries <= (double)(int64_t(1) << 32) ? 1 : 0;
        case POT_PCOST_ON_THE_FLY: return 0;
        case POT_PCOST_KEEP: return entries <= (double)(int64_t(1) << 36) ? 1 : -1;
        default: return -1;
    }
}

Layout plan_of(const pot_clouds *c) {
    return plan(c->n, c->m, c->d, c->precision, c->cost_p, c->cmat != nullptr);
}

bool valid_sizes(int64_t n, int64_t m, int32_t d, int32_t precision) {
    return n >= 1 && m >= 1 && d >= 1 && d <= POT_MAX_D &&
           (precision == POT_PREC_FP32 || precision == POT_PREC_BF16 ||
            precision == POT_PREC_BF16X3) &&
           n <= (int64_t(1) << 31) && m <= (int64_t(1) << 31);
}

bool valid_clouds(const pot_clouds *c) {
    if (!c || !c->ws || !c->X || !c->Y || !c->xk) return false;
    if (!valid_sizes(c->n, c->m, c->d, c->precision) || !valid_cost_p(c->cost_p)) return false;
    if (c->precision != POT_PREC_FP32 && (!c->x_lp || !c->y_lp || !c->yt_lp)) return false;
    if (c->cost_p != 0.f &&
        (c->precision != POT_PREC_FP32 ||
         (c->cmat ? c->ldc != pot::pcost_ldc(c->m) : c->ldc != 0)))
        return false;
    return c->ws_bytes >= plan_of(c).total;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void bind_clouds(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                 const float *a, const float *b, int32_t precision, void *ws, size_t ws_bytes,
                 const Layout &L, float cost_p, bool keep_cost) {
    std::memset(c, 0, sizeof(*c));
    c->n = n; c->m = m; c->d = d; c->precision = precision;
    c->X = X; c->Y = Y; c->a = a; c->b = b; c->ws = ws; c->ws_bytes = ws_bytes;
    c->xk = at<float>(c, L.xk);
    c->x_sqn = at<float>(c, L.xsq);
    c->y_sqn = at<float>(c, L.ysq);
    c->log_a = at<float>(c, L.la);
    c->log_b = at<float>(c, L.lb);
    c->x_lp = precision != POT_PREC_FP32 ? at<void>(c, L.xlp) : nullptr;
    c->y_lp = precision != POT_PREC_FP32 ? at<void>(c, L.ylp) : nullptr;
    c->yt_lp = precision != POT_PREC_FP32 ? at<void>(c, L.ytl) : nullptr;
    c->cost_p = cost_p;
    c->cmat = cost_p != 0.f && keep_cost ? at<float>(c, L.cm) : nullptr;
    c->ldc = c->cmat ? pot::pcost_ldc(m) : 0;
}

int refresh_pcost(pot_clouds *c, const Layout &L, hipStream_t s) {
    double *part = at<double>(c, L.cmp);
    const int64_t nb = pot::pcost_matrix_blocks(c->n, c->m);
    POT_TRY(pot::launch_pcost_matrix(c->xk, c->n, c->Y, c->m, c->d, c->cost_p, c->cmat, c->ldc, part,
                                     part + nb, s));
    double sum = 0.0;
    POT_TRY(hipMemcpyAsync(&sum, part + nb, sizeof(double), hipMemcpyDeviceToHost, s));
    POT_TRY(hipStreamSynchronize(s));
    c->mean_cost = sum / ((double)c->n * (double)c->m);
    return std::isfinite(c->mean_cost) ? POT_OK : POT_ERR_NUMERIC;
}

bool map_writes_norms(const pot_clouds *c) {
    return c->precision == POT_PREC_FP32 && c->cost_p == 0.f;
}

int enqueue_moments(pot_clouds *c, const Layout &L, double *host, hipStream_t s, bool norms_ready) {
    const int d = c->d;
    POT_TRY(pot::launch_cloud_prep(c->xk, c->n, d, c->x_sqn, c->x_lp, at<double>(c, L.xst),
                                   pot::cloud_stat_blocks(c->n), s, norms_ready));
    POT_TRY(hipMemcpyAsync(host, at<double>(c, L.xst), (d + 1) * 8, hipMemcpyDeviceToHost, s));
    POT_TRY(hipMemcpyAsync(host + d + 1, at<double>(c, L.yst), (d + 1) * 8, hipMemcpyDeviceToHost, s));
    return POT_OK;
}

int enqueue_prepare(pot_clouds *c, const Layout &L, double *host, hipStream_t s) {
    POT_TRY(hipMemcpyAsync(c->xk, c->X, (size_t)c->n * c->d * sizeof(float), hipMemcpyDeviceToDevice, s));
    POT_TRY(pot::launch_log_weights(c->a, c->n, c->log_a, s));
    POT_TRY(pot::launch_log_weights(c->b, c->m, c->log_b, s));
    POT_TRY(pot::launch_cloud_prep(c->Y, c->m, c->d, c->y_sqn, c->y_lp, at<double>(c, L.yst),
                                   pot::cloud_stat_blocks(c->m), s));
    if (c->yt_lp) {
        if (c->precision == POT_PREC_BF16)
            POT_TRY(pot::launch_f16_transpose(c->Y, c->m, c->d, c->yt_lp, at<float>(c, L.yts), s));
        else
            POT_TRY(pot::launch_bf16_transpose(c->Y, c->m, c->d, c->yt_lp, s));
    }
    return enqueue_moments(c, L, host, s);
}

int finish_moments(pot_clouds *c, const double *host) {
    const int d = c->d;
    const double *sx = host, *sy = host + d + 1;
    const double n = (double)c->n, m = (double)c->m;
    double dot = 0.0;
    for (int k = 0; k < d; ++k) dot += (sx[k] / n) * (sy[k] / m);
    c->mean_cost = sx[d] / n + sy[d] / m - 2.0 * dot;
    return std::isfinite(c->mean_cost) ? POT_OK : POT_ERR_NUMERIC;
}

LseJob f_job(const pot_clouds *c, const Layout &L, float eps) {
    LseJob a{};
    a.U = c->xk; a.U_lp = c->x_lp; a.nu = c->n; a.usq = c->x_sqn; a.logw = c->log_a;
    a.V = c->Y; a.V_lp = c->y_lp; a.nv = c->m; a.vsq = c->y_sqn;
    a.eps = eps; a.d = c->d; a.precision = c->precision; a.gamma = 1.f;
    a.part_m = at<float>(c, L.pm); a.part_s = at<float>(c, L.ps); a.err_part = at<float>(c, L.errp);
    if (c->cost_p != 0.f) { a.cost_p = c->cost_p; a.cmat = c->cmat; a.ldc = c->ldc; a.cmat_cols = 0; a.usq = nullptr; }
    return a;
}

LseJob g_job(const pot_clouds *c, const Layout &L, float eps) {
    LseJob a{};
    a.U = c->Y; a.U_lp = c->y_lp; a.nu = c->m; a.usq = c->y_sqn; a.logw = c->log_b;
    a.V = c->xk; a.V_lp = c->x_lp; a.nv = c->n; a.vsq = c->x_sqn;
    a.eps = eps; a.d = c->d; a.precision = c->precision; a.gamma = 1.f;
    a.part_m = at<float>(c, L.pm); a.part_s = at<float>(c, L.ps); a.err_part = nullptr;
    if (c->cost_p != 0.f) { a.cost_p = c->cost_p; a.cmat = c->cmat; a.ldc = c->ldc; a.cmat_cols = 1; a.usq = nullptr; }
    return a;
}

void alpha_schedule(int K, int kind, float *alpha) {
    for (int k = 0; k < K; ++k) {
        double a;
        if (kind == 1) {
            a = 1.0 / std::exp(1.0);
        } else {
            const double tk = kind == 2 ? std::pow((double)k / K, 2.0) : (double)k / K;
            const double t1 = kind == 2 ? std::pow((double)(k + 1) / K, 2.0) : (double)(k + 1) / K;
            a = (t1 - tk) / (1.0 - tk);
        }
        alpha[k] = (float)a;
    }
    alpha[K - 1] = 1.f;
}

bool valid_params(const pot_progot_params *p) {
    if (!p || p->K < 1 || p->K > POT_MAX_K || p->max_iter < 1 || p->alpha_sched < 0 ||
        p->alpha_sched > 2)
        return false;
    if (p->eps_mode == 0) {
        if (!finite_pos(p->theta)) return false;
    } else if (p->eps_mode == 1) {
        if (!p->eps_explicit) return false;
        for (int k = 0; k < p->K; ++k)
            if (!(p->eps_explicit[k] > 0.0) || !std::isfinite(p->eps_explicit[k])) return false;
    } else {
        return false;
    }
    return p->tau_first >= 0.f && p->tau_last >= 0.f && std::isfinite(p->tau_first) &&
           std::isfinite(p->tau_last);
}

int step_values(const pot_progot_params *p, const float *alpha, int k, double mean_cost,
                float *eps, float *tau, float *gamma) {
    const int K = p->K;
    *eps = p->eps_mode == 0 ? (float)(p->theta * mean_cost / 20.0) : (float)p->eps_explicit[k];
    if (!finite_pos(*eps)) return POT_ERR_NUMERIC;
    *tau = K == 1 ? p->tau_last
                  : p->tau_first + (p->tau_last - p->tau_first) * (float)k / (float)(K - 1);
    const float w = (p->warm_start == 0 || k == 0) ? alpha[k] : alpha[k - 1];
    *gamma = 1.f - w;
    return POT_OK;
}

int run_map(const pot_clouds *c, const float *g, float eps, const float *Xq, int64_t nq,
            float alpha, float *Xout, hipStream_t s, float *out_sqn) {
    if (c->cost_p != 0.f) {
        const Layout L = plan_of(c);
        pot::PcostMapArgs a{};
        a.Xq = Xq; a.nq = nq; a.Y = c->Y; a.m = c->m; a.g = g;
        a.eps = eps; a.alpha = alpha; a.p = c->cost_p; a.d = c->d; a.Xout = Xout;
        a.pm = at<float>(c, L.pm); a.ps = at<float>(c, L.ps); a.pacc = at<float>(c, L.mpa);
        a.cap_q = c->n;
        POT_TRY(pot::launch_pcost_map(a, s));
        return POT_OK;
    }
    MapArgs a{};
    a.Xq = Xq; a.nq = nq; a.Y = c->Y; a.Y_lp = c->y_lp; a.m = c->m; a.ysq = c->y_sqn; a.g = g;
    a.eps = eps; a.alpha = alpha; a.d = c->d; a.precision = c->precision;
    a.YT_lp = c->yt_lp; a.mp = pot::bf16_mpad(c->m);
    a.yt_unscale = c->precision == POT_PREC_BF16 ? at<float>(c, plan_of(c).yts) + 1 : nullptr;
    a.Xout = Xout; a.out_sqn = map_writes_norms(c) ? out_sqn : nullptr;
    POT_TRY(pot::launch_entropic_map(a, s));
    return POT_OK;
}

}  // namespace host
}  // namespace pot

namespace {

using namespace pot::host;
using pot::LseJob;

// Per-thread pinned landing zone for scalar read-backs: coherent host memory
// mapped into the device's address space, so the kernel that forms a scalar
// (an error sum) stores it there itself and the host reads it once an event
// after that kernel has completed; no copy command per read-back.
// The Sinkhorn loop returns while up to two iterations past the returned one
// may still be queued (the entry points synchronise their stream before they
// return, but an error return or an internal caller need not), and their
// error sums land in these slots; `tail` marks the end of the last solve's
// work on `tail_stream`, and a solve on another stream waits for it before it
// reuses the slots.
struct Pinned {
    float *buf = nullptr;
    float *dev = nullptr;   // the same memory, as the device addresses it
    hipEvent_t tail = nullptr;
    hipStream_t tail_stream = nullptr;
    bool tail_set = false;
    ~Pinned() {
        if (tail) (void)hipEventDestroy(tail);
        if (buf) (void)hipHostFree(buf);
    }
};
thread_local Pinned g_pinned;

// Claims the pinned slots for a solve on stream s (see Pinned) and, on
// destruction, marks the end of the work it enqueued.
struct SlotClaim {
    hipStream_t s;
    bool ok = false;
    bool inert = false;   // the solve does not use the pinned slots
    explicit SlotClaim(hipStream_t st, bool unused = false) : s(st), inert(unused) {
        if (inert) { ok = true; return; }
        if (!g_pinned.tail && hipEventCreateWithFlags(&g_pinned.tail, hipEventDisableTiming) != hipSuccess) {
            g_pinned.tail = nullptr;
            return;
        }
        if (g_pinned.tail_set && g_pinned.tail_stream != s && hipEventSynchronize(g_pinned.tail) != hipSuccess)
            return;
        ok = true;
    }
    ~SlotClaim() {
        if (!ok || inert) return;
        g_pinned.tail_set = hipEventRecord(g_pinned.tail, s) == hipSuccess;
        g_pinned.tail_stream = s;
    }
};

float *pinned_slot(float **dev) {
    if (!g_pinned.buf) {
        if (hipHostMalloc(reinterpret_cast<void **>(&g_pinned.buf), 64 * sizeof(float),
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            g_pinned.buf = nullptr;
            return nullptr;
        }
        if (hipHostGetDevicePointer(reinterpret_cast<void **>(&g_pinned.dev), g_pinned.buf, 0) !=
            hipSuccess) {
            (void)hipHostFree(g_pinned.buf);
            g_pinned.buf = g_pinned.dev = nullptr;
            return nullptr;
        }
    }
    *dev = g_pinned.dev;
    return g_pinned.buf;
}

// Synchronous mean-cost refresh of the source iterate (single-problem path);
// for a general cost, the cost matrix is rebuilt with it.  norms_ready: the
// map that moved the iterate wrote its squared norms.
int refresh_mean_cost(pot_clouds *c, const Layout &L, hipStream_t s, bool norms_ready = false) {
    if (c->cost_p != 0.f) return refresh_pcost(c, L, s);
    std::vector<double> host(moments_len(c->d));
    int st = enqueue_moments(c, L, host.data(), s, norms_ready);
    if (st != POT_OK) return st;
    POT_TRY(hipStreamSynchronize(s));
    return finish_moments(c, host.data());
}

struct SinkResult {
    int iters = 0;
    float err = 0.f;
    bool converged = false;
    const float *f = nullptr, *g = nullptr;
};

// Enqueue err = sum of the error partials into a pinned slot (`slot`, its
// device address), unless a later update already carries it (summed = true),
// and the event the host waits on before reading the slot.
int enqueue_err_readback(const pot_clouds *c, const Layout &L, int nparts, float *slot,
                         hipEvent_t ev, hipStream_t s, bool summed = false) {
    if (!summed) POT_TRY(pot::launch_sum_f32(at<float>(c, L.errp), nparts, slot, s));
    if (ev) POT_TRY(hipEventRecord(ev, s));
    return POT_OK;
}

// Alg. 1 on c->xk.  Iteration t: f_t from g_{t-1} (whose error partials are
// the row-marginal error of iterate t-1), then g_t from f_t.  The host reads
// err(t-1) back with a lag chosen from the cost of one iteration:
//   lag 2 (cheap iterations): err(t-2) is checked after g_t is enqueued, so
//         the stream always holds the next iterations while the host waits
//         and no time is lost between launches;
//   lag 1: err(t-1) is checked after g_t is enqueued (g_t runs while the
//         host waits; one iteration past convergence is computed);
//   lag 0 (iterations of a millisecond or more): err(t-1) is checked before
//         g_t is enqueued, so no g-update past convergence is computed; the
//         host's reaction time is small beside the iteration.
// The potentials live in a ring of three slots, so the iterate whose error
// is being read is still intact when it is returned.  Errors are checked in
// order and the first iterate with err <= tau is returned in every mode.
// At lag 2, where the g-update's kernel can carry it (the general-cost
// column kernel), the sum of f_t's error partials rides in g_t's first
// workgroup instead of a launch of its own; the copy then follows g_t, which
// the host does not wait for until two iterations later.
constexpr int kRing = 3;

int pick_lag(const pot_clouds *c) {
    const double nm = (double)c->n * (double)c->m;
    double us;   // estimated time of one iteration (two potential updates)
    if (c->cost_p != 0.f) {
        us = 2.0 * nm * 4.0 / 5e12 * 1e6;                 // the cost matrix read twice
    } else {
        const double rate = c->precision == POT_PREC_FP32 ? 110e12
                          : c->precision == POT_PREC_BF16 ? 900e12 : 400e12;
        us = 4.0 * nm * c->d / rate * 1e6;                 // 2 n m d flops per update
    }
    return us < 100.0 ? 2 : us < 1000.0 ? 1 : 0;
}

struct Events {
    hipEvent_t ev[kRing] = {};
    ~Events() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// copy_rb: the error sums go to device slots in the workspace and each check
// copies one back and synchronises the stream (lag 0); no pinned host memory
// and no events are created, for the entry points that allocate nothing.
// The iterates and the returned one are the same as with the mapped slots.
int sinkhorn_core(const pot_clouds *c, const Layout &L, float eps, float tau, int max_iter,
                  const float *g_init, float gamma, SinkResult *out, hipStream_t s,
                  bool copy_rb = false, const float *f_warm = nullptr) {
    float *fb[kRing] = {at<float>(c, L.f0), at<float>(c, L.f1), at<float>(c, L.f2)};
    float *gb[kRing] = {at<float>(c, L.g0), at<float>(c, L.g1), at<float>(c, L.g2)};
    float *hdev = nullptr;
    float *host = nullptr;
    if (copy_rb) {
        hdev = at<float>(c, L.eslot);
    } else {
        host = pinned_slot(&hdev);
        if (!host) return POT_ERR_DEVICE;
    }
    SlotClaim claim(copy_rb ? nullptr : s, copy_rb);
    if (!claim.ok) return POT_ERR_DEVICE;
    Events E;
    if (!copy_rb)
        for (hipEvent_t &e : E.ev) POT_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const int lag = copy_rb ? 0 : pick_lag(c);
    LseJob fa = f_job(c, L, eps);
    LseJob ga = g_job(c, L, eps);
    const bool fold = lag == 2 && pot::lse_update_folds_sum(ga);
    // read err_k (its sum was enqueued with f_{k+1}, or rides in g_{k+1}); true when the loop ends at k
    float copied = 0.f;
    auto read_err = [&](int k) -> bool {
        if (copy_rb)
            return hipMemcpyAsync(&copied, hdev + k % kRing, sizeof(float), hipMemcpyDeviceToHost, s) ==
                       hipSuccess &&
                   hipStreamSynchronize(s) == hipSuccess;
        if (hipEventSynchronize(E.ev[k % kRing]) != hipSuccess) return false;
        copied = host[k % kRing];
        return true;
    };
    auto check = [&](int k, int *status) -> bool {
        if (!read_err(k)) { *status = POT_ERR_DEVICE; return true; }
        const float err = copied;
        if (!std::isfinite(err)) { *status = POT_ERR_NUMERIC; return true; }
        if (tau > 0.f && err <= tau) {
            out->iters = k; out->err = err; out->converged = true;
            out->f = fb[k % kRing]; out->g = gb[k % kRing];
            return true;
        }
        return false;
    };
    int status = POT_OK;
    for (int t = 1;; ++t) {
        fa.vpot = t == 1 ? g_init : gb[(t - 1) % kRing];
        fa.gamma = t == 1 ? gamma : 1.f;
        fa.pot_old = t == 1 ? nullptr : fb[(t - 1) % kRing];
        fa.shift_pot = t == 1 ? f_warm : fa.pot_old;
        fa.shift_gamma = t == 1 ? gamma : 1.f;
        fa.pot_out = fb[t % kRing];
        int nparts = 0;
        if (pot::launch_lse_update(fa, s, &nparts) != hipSuccess) return POT_ERR_DEVICE;
        if (t > 1 && !fold &&
            (status = enqueue_err_readback(c, L, nparts, hdev + (t - 1) % kRing, E.ev[(t - 1) % kRing],
                                           s)) != POT_OK)
            return status;
        if (lag == 0 && t > 1 && check(t - 1, &status)) return status;
        ga.vpot = fb[t % kRing];
        ga.shift_pot = t == 1 ? g_init : gb[(t - 1) % kRing];
        ga.shift_gamma = t == 1 ? gamma : 1.f;
        ga.pot_out = gb[t % kRing];
        const bool carry = fold && t > 1;
        ga.esum_in = carry ? at<float>(c, L.errp) : nullptr;
        ga.esum_n = carry ? nparts : 0;
        ga.esum_out = carry ? hdev + (t - 1) % kRing : nullptr;
        if (pot::launch_lse_update(ga, s, nullptr) != hipSuccess) return POT_ERR_DEVICE;
        if (carry && (status = enqueue_err_readback(c, L, nparts, hdev + (t - 1) % kRing,
                                                    E.ev[(t - 1) % kRing], s, true)) != POT_OK)
            return status;
        // err_{t-lag}: its slots are not written before iteration t + 1
        if (lag > 0 && t - lag >= 1 && check(t - lag, &status)) return status;
        if (t == max_iter) {
            for (int k = std::max(1, t - lag + 1); k < t; ++k)
                if (check(k, &status)) return status;
            // err of the last iterate: one more f-update into the free slot
            fa.vpot = gb[t % kRing]; fa.gamma = 1.f;
            fa.pot_old = fb[t % kRing]; fa.shift_pot = fa.pot_old; fa.shift_gamma = 1.f;
            fa.pot_out = fb[(t + 1) % kRing];
            if (pot::launch_lse_update(fa, s, &nparts) != hipSuccess) return POT_ERR_DEVICE;
            if ((status = enqueue_err_readback(c, L, nparts, hdev + t % kRing, E.ev[t % kRing], s)) !=
                POT_OK)
                return status;
            if (check(t, &status)) return status;
            out->iters = t; out->err = copied;
            out->converged = tau > 0.f ? out->err <= tau : true;
            out->f = fb[t % kRing]; out->g = gb[t % kRing];
            return POT_OK;
        }
    }
}

}  // namespace

namespace pot {
namespace host {

int run_sinkhorn(const pot_clouds *c, const Layout &L, float eps, float tau, int max_iter,
                 const float *g_init, float gamma, SinkOut *out, hipStream_t s) {
    SinkResult r;
    const int st = sinkhorn_core(c, L, eps, tau, max_iter, g_init, gamma, &r, s);
    out->iters = r.iters; out->err = r.err; out->converged = r.converged;
    out->f = r.f; out->g = r.g;
    return st;
}

}  // namespace host
}  // namespace pot

extern "C" {

const char *pot_status_string(int code) {
    switch (code) {
        case POT_OK: return "ok";
        case POT_WARN_NOT_CONVERGED: return "not converged: max_iter reached with err > tau";
        case POT_BUSY: return "busy: not admitted now or still in flight";
        case POT_ERR_INVALID: return "invalid argument";
        case POT_ERR_NOMEM: return "workspace too small";
        case POT_ERR_NUMERIC: return "non-finite marginal error or mean cost";
        case POT_ERR_DEVICE: return "HIP runtime error";
        default: return "unknown status";
    }
}

const char *pot_version(void) { return "0.1.0"; }

size_t pot_workspace_bytes(int64_t n, int64_t m, int32_t d, int32_t precision) {
    if (!valid_sizes(n, m, d, precision)) return 0;
    return plan(n, m, d, precision).total;
}

}  // extern "C"

namespace {

// Weights, when given, must be positive and sum to 1 within 1e-5.  They are
// read back in chunks through a buffer on the stack (no host allocation).
int check_weights(const float *a, int64_t n, const float *b, int64_t m, hipStream_t s) {
    constexpr int64_t kChunk = 8192;
    float h[kChunk];
    for (int side = 0; side < 2; ++side) {
        const float *w = side ? b : a;
        const int64_t len = side ? m : n;
        if (!w) continue;
        double tot = 0.0;
        for (int64_t i0 = 0; i0 < len; i0 += kChunk) {
            const int64_t cnt = std::min(kChunk, len - i0);
            POT_TRY(hipMemcpyAsync(h, w + i0, cnt * sizeof(float), hipMemcpyDeviceToHost, s));
            POT_TRY(hipStreamSynchronize(s));
            for (int64_t i = 0; i < cnt; ++i) {
                if (!(h[i] > 0.f) || !std::isfinite(h[i])) return POT_ERR_INVALID;
                tot += h[i];
            }
        }
        if (std::fabs(tot - 1.0) > 1e-5) return POT_ERR_INVALID;
    }
    return POT_OK;
}

int prepare(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
            const float *a, const float *b, int32_t precision, float cost_p, bool keep, void *ws,
            size_t ws_bytes, hipStream_t s) {
    const Layout L = plan(n, m, d, precision, cost_p, keep);
    if (ws_bytes < L.total) return POT_ERR_NOMEM;
    int st = check_weights(a, n, b, m, s);
    if (st != POT_OK) return st;
    bind_clouds(c, X, n, Y, m, d, a, b, precision, ws, ws_bytes, L, cost_p, keep);
    double host[2 * (POT_MAX_D + 1)];   // moments_len(d) <= this
    if ((st = enqueue_prepare(c, L, host, s)) != POT_OK) return st;
    POT_TRY(hipStreamSynchronize(s));
    if ((st = finish_moments(c, host)) != POT_OK) return st;
    return cost_p != 0.f ? refresh_pcost(c, L, s) : POT_OK;
}

bool valid_pcost_sizes(int64_t n, int64_t m, int32_t d, float p, int32_t flags) {
    return p != 0.f && valid_cost_p(p) && valid_sizes(n, m, d, POT_PREC_FP32) &&
           pcost_keep(n, m, flags) >= 0 && pot::pcost_matrix_blocks(n, m) <= 0x7fffffff;
}

}  // namespace

extern "C" {

int pot_prepare_clouds(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m,
                       int32_t d, const float *a, const float *b, int32_t precision, void *ws,
                       size_t ws_bytes, void *stream) {
    if (!c || !X || !Y || !ws || !valid_sizes(n, m, d, precision)) return POT_ERR_INVALID;
    return prepare(c, X, n, Y, m, d, a, b, precision, 0.f, true, ws, ws_bytes,
                   static_cast<hipStream_t>(stream));
}

size_t pot_workspace_bytes_pcost(int64_t n, int64_t m, int32_t d, float p, int32_t flags) {
    if (!valid_pcost_sizes(n, m, d, p, flags)) return 0;
    return plan(n, m, d, POT_PREC_FP32, p, pcost_keep(n, m, flags) == 1).total;
}

int pot_prepare_clouds_pcost(pot_clouds *c, const float *X, int64_t n, const float *Y, int64_t m,
                             int32_t d, const float *a, const float *b, float p, int32_t flags,
                             void *ws, size_t ws_bytes, void *stream) {
    if (!c || !X || !Y || !ws || !valid_pcost_sizes(n, m, d, p, flags)) return POT_ERR_INVALID;
    return prepare(c, X, n, Y, m, d, a, b, POT_PREC_FP32, p, pcost_keep(n, m, flags) == 1, ws,
                   ws_bytes, static_cast<hipStream_t>(stream));
}

int pot_sinkhorn_solve(pot_clouds *c, float eps, float tau, int32_t max_iter, const float *f_init,
                       const float *g_init, float *f, float *g, pot_sinkhorn_info *info,
                       void *stream) {
    (void)f_init;  // the first f-update overwrites f (Alg. 1): f_init cannot matter
    if (!valid_clouds(c) || !f || !g || !finite_pos(eps) || !(tau >= 0.f) || !std::isfinite(tau) ||
        max_iter < 1)
        return POT_ERR_INVALID;
    const double t0 = now_s();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = plan_of(c);
    SinkResult r;
    int st = sinkhorn_core(c, L, eps, tau, max_iter, g_init, 1.f, &r, s);
    if (st != POT_OK) return st;
    POT_TRY(hipMemcpyAsync(f, r.f, c->n * sizeof(float), hipMemcpyDeviceToDevice, s));
    POT_TRY(hipMemcpyAsync(g, r.g, c->m * sizeof(float), hipMemcpyDeviceToDevice, s));
    POT_TRY(hipStreamSynchronize(s));
    if (info) {
        info->iters = r.iters; info->converged = r.converged ? 1 : 0; info->err = r.err;
        info->seconds = now_s() - t0;
    }
    return r.converged ? POT_OK : POT_WARN_NOT_CONVERGED;
}

int pot_entropic_map(const pot_clouds *c, const float *g, float eps, const float *Xq, int64_t nq,
                     float alpha, float *Xout, void *stream) {
    if (!valid_clouds(c) || !g || !finite_pos(eps) || nq < 0 || !(alpha >= 0.f && alpha <= 1.f))
        return POT_ERR_INVALID;
    if (nq == 0) return POT_OK;
    if (!Xq || !Xout || nq > (int64_t(1) << 31)) return POT_ERR_INVALID;
    return run_map(c, g, eps, Xq, nq, alpha, Xout, static_cast<hipStream_t>(stream));
}

int pot_progot_solve(pot_clouds *c, const pot_progot_params *p, float *f, float *G, float *TX,
                     pot_progot_info *info, void *stream) {
    if (!valid_clouds(c) || !valid_params(p) || !f || !G) return POT_ERR_INVALID;
    const double t0 = now_s();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = plan_of(c);
    const int K = p->K;
    const int64_t n = c->n, m = c->m;
    float alpha[POT_MAX_K];
    alpha_schedule(K, p->alpha_sched, alpha);

    POT_TRY(hipMemcpyAsync(c->xk, c->X, (size_t)n * c->d * sizeof(float), hipMemcpyDeviceToDevice, s));
    int st = refresh_mean_cost(c, L, s);
    if (st != POT_OK) return st;

    pot_progot_info loc{};
    loc.K = K;
    loc.converged = 1;
    const float *f_prev = nullptr;   // the previous step's f (a ring slot of the workspace)
    for (int k = 0; k < K; ++k) {
        float eps, tau, gamma;
        st = step_values(p, alpha, k, c->mean_cost, &eps, &tau, &gamma);
        if (st != POT_OK) return st;
        const float *g_init = k == 0 ? nullptr : G + (size_t)(k - 1) * m;
        SinkResult r;
        // the warm start of both potentials also serves as the exponent
        // shift of the first iteration (BF16 forms)
        st = sinkhorn_core(c, L, eps, tau, p->max_iter, g_init, gamma, &r, s, false, f_prev);
        if (st != POT_OK) return st;
        f_prev = r.f;
        POT_TRY(hipMemcpyAsync(G + (size_t)k * m, r.g, m * sizeof(float), hipMemcpyDeviceToDevice, s));
        loc.iters[k] = r.iters; loc.err[k] = r.err; loc.eps[k] = eps; loc.alpha[k] = alpha[k];
        if (!r.converged) loc.converged = 0;
        if (k + 1 < K) {
            st = run_map(c, G + (size_t)k * m, eps, c->xk, n, alpha[k], c->xk, s, c->x_sqn);
            if (st != POT_OK) return st;
            // norms (unless the map wrote them), BF16 copy and mean cost of X^(k+1)
            st = refresh_mean_cost(c, L, s, map_writes_norms(c));
            if (st != POT_OK) return st;
        } else {
            POT_TRY(hipMemcpyAsync(f, r.f, n * sizeof(float), hipMemcpyDeviceToDevice, s));
            if (TX) {
                st = run_map(c, G + (size_t)k * m, eps, c->xk, n, 1.f, TX, s);
                if (st != POT_OK) return st;
            }
        }
    }
    POT_TRY(hipStreamSynchronize(s));
    loc.seconds = now_s() - t0;
    if (info) *info = loc;
    return loc.converged ? POT_OK : POT_WARN_NOT_CONVERGED;
}

int pot_progot_map(const pot_clouds *c, int32_t K, const float *G, const float *eps,
                   const float *alpha, const float *Xq, int64_t nq, float *Yout, void *stream) {
    if (!valid_clouds(c) || K < 1 || K > POT_MAX_K || !G || !eps || !alpha || nq < 0)
        return POT_ERR_INVALID;
    for (int k = 0; k < K; ++k) {
        if (!finite_pos(eps[k])) return POT_ERR_INVALID;
        if (k + 1 < K && !(alpha[k] >= 0.f && alpha[k] <= 1.f)) return POT_ERR_INVALID;
    }
    if (nq == 0) return POT_OK;
    if (!Xq || !Yout || nq > (int64_t(1) << 31)) return POT_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (int k = 0; k < K; ++k) {
        const float a = k + 1 == K ? 1.f : alpha[k];
        const int st = run_map(c, G + (size_t)k * c->m, eps[k], k == 0 ? Xq : Yout, nq, a, Yout, s);
        if (st != POT_OK) return st;
    }
    return POT_OK;
}

int pot_coupling_metrics(const pot_clouds *c, const float *f, const float *g, float eps,
                         double *out, void *stream) {
    if (!valid_clouds(c) || !f || !g || !out || !finite_pos(eps)) return POT_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = plan_of(c);
    const int nbr = pot::fp64_check_blocks(c->n), nbc = pot::fp64_check_blocks(c->m);
    constexpr int Q = pot::kCheckParts;
    if (c->cost_p != 0.f)
        POT_TRY(pot::launch_fp64_check_pcost(c->xk, c->n, c->Y, c->m, c->d, c->cost_p, f, g, c->a,
                                             c->b, eps, at<double>(c, L.chr), at<double>(c, L.chc), s));
    else
        POT_TRY(pot::launch_fp64_check(c->xk, c->n, c->Y, c->m, c->d, f, g, c->a, c->b, eps,
                                       at<double>(c, L.n64), at<double>(c, L.n64) + c->n,
                                       at<double>(c, L.chr), at<double>(c, L.chc), s));
    std::vector<double> hr(Q * (size_t)nbr), hc(Q * (size_t)nbc);
    POT_TRY(hipMemcpyAsync(hr.data(), at<double>(c, L.chr), hr.size() * 8, hipMemcpyDeviceToHost, s));
    POT_TRY(hipMemcpyAsync(hc.data(), at<double>(c, L.chc), hc.size() * 8, hipMemcpyDeviceToHost, s));
    POT_TRY(hipStreamSynchronize(s));
    double row = 0, mass = 0, fa = 0, pc = 0, plp = 0, col = 0, gb = 0;
    for (int b = 0; b < nbr; ++b) {
        row += hr[Q * b]; mass += hr[Q * b + 1]; fa += hr[Q * b + 2];
        pc += hr[Q * b + 3]; plp += hr[Q * b + 4];
    }
    for (int b = 0; b < nbc; ++b) { col += hc[Q * b]; gb += hc[Q * b + 2]; }
    out[0] = row;
    out[1] = col;
    out[2] = fa + gb - (double)eps * mass;
    out[3] = pc;
    out[4] = plp;
    out[5] = mass;
    if (!std::isfinite(row) || !std::isfinite(col)) return POT_ERR_NUMERIC;
    return POT_OK;
}

int pot_marginal_check(const pot_clouds *c, const float *f, const float *g, float eps, double *out,
                       void *stream) {
    if (!out) return POT_ERR_INVALID;
    double m6[6];
    const int st = pot_coupling_metrics(c, f, g, eps, m6, stream);
    if (st == POT_OK || st == POT_ERR_NUMERIC) { out[0] = m6[0]; out[1] = m6[1]; out[2] = m6[2]; }
    return st;
}

size_t pot_sinkhorn_divergence_bytes(int64_t n, int64_t m, int32_t d) {
    if (!valid_sizes(n, m, d, POT_PREC_FP32)) return 0;
    return std::max({plan(n, m, d, POT_PREC_FP32).total, plan(n, n, d, POT_PREC_FP32).total,
                     plan(m, m, d, POT_PREC_FP32).total});
}

size_t pot_sinkhorn_divergence_pcost_bytes(int64_t n, int64_t m, int32_t d, float p) {
    const int32_t A = POT_PCOST_AUTO;
    if (!valid_pcost_sizes(n, m, d, p, A) || !valid_pcost_sizes(n, n, d, p, A) ||
        !valid_pcost_sizes(m, m, d, p, A))
        return 0;
    return std::max({plan(n, m, d, POT_PREC_FP32, p, pcost_keep(n, m, A) == 1).total,
                     plan(n, n, d, POT_PREC_FP32, p, pcost_keep(n, n, A) == 1).total,
                     plan(m, m, d, POT_PREC_FP32, p, pcost_keep(m, m, A) == 1).total});
}

}  // extern "C"

namespace {

// eq. sink_div: the pairs (Y, Y), (X, Y), (X, X) solved one after another in
// the same workspace; (Y, Y) first, whose mean cost gives the default
// eps_D = 5 % of the mean cost within Y.
int divergence(const float *X, int64_t n, const float *Y, int64_t m, int32_t d, const float *a,
               const float *b, float cost_p, float eps, float tau, int32_t max_iter, double *out,
               void *ws, size_t ws_bytes, hipStream_t s, bool noalloc = false) {
    struct Pair { const float *U; int64_t nu; const float *wu; const float *V; int64_t nv; const float *wv; };
    const Pair pairs[3] = {{Y, m, b, Y, m, b}, {X, n, a, Y, m, b}, {X, n, a, X, n, a}};
    double ot[3];
    bool all = true;
    for (int k = 0; k < 3; ++k) {
        const Pair &q = pairs[k];
        const bool keep = cost_p == 0.f || pcost_keep(q.nu, q.nv, POT_PCOST_AUTO) == 1;
        const Layout L = plan(q.nu, q.nv, d, POT_PREC_FP32, cost_p, keep);
        pot_clouds c;
        int st = prepare(&c, q.U, q.nu, q.V, q.nv, d, q.wu, q.wv, POT_PREC_FP32, cost_p, keep, ws, L.total,
                         s);
        if (st != POT_OK) return st;
        if (k == 0 && eps == 0.f) eps = (float)(0.05 * c.mean_cost);
        if (!finite_pos(eps)) return POT_ERR_NUMERIC;
        SinkResult r;
        if ((st = sinkhorn_core(&c, L, eps, tau, max_iter, nullptr, 1.f, &r, s, noalloc)) != POT_OK)
            return st;
        all = all && r.converged;
        // The returned iterate ends with a g-update, so its coupling's column
        // sums are b and its mass sum_ij P_ij is 1: the objective of eq.
        // entdual is <f, a> + <g, b> - eps, two FP64 dot products (the FP64
        // pass over all pairs would add only rounding of the FP32 g).
        double *part = at<double>(&c, L.n64);   // >= 512 doubles
        const int nbf = pot::weighted_sum_blocks(q.nu), nbg = pot::weighted_sum_blocks(q.nv);
        POT_TRY(pot::launch_weighted_sum(r.f, q.wu, q.nu, part, s));
        POT_TRY(pot::launch_weighted_sum(r.g, q.wv, q.nv, part + 256, s));
        double h[512];
        POT_TRY(hipMemcpyAsync(h, part, sizeof(double) * 512, hipMemcpyDeviceToHost, s));
        POT_TRY(hipStreamSynchronize(s));
        double fa = 0.0, gb = 0.0;
        for (int b2 = 0; b2 < nbf; ++b2) fa += h[b2];
        for (int b2 = 0; b2 < nbg; ++b2) gb += h[256 + b2];
        ot[k] = fa + gb - (double)eps;
        if (!std::isfinite(ot[k])) return POT_ERR_NUMERIC;
    }
    out[0] = ot[1] - 0.5 * (ot[2] + ot[0]);
    out[1] = ot[1];
    out[2] = ot[2];
    out[3] = ot[0];
    out[4] = (double)eps;
    return all ? POT_OK : POT_WARN_NOT_CONVERGED;
}

}  // namespace

extern "C" {

int pot_sinkhorn_divergence(const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                            const float *a, const float *b, float eps, float tau, int32_t max_iter,
                            double *out, void *ws, size_t ws_bytes, void *stream) {
    if (!X || !Y || !out || !ws || !valid_sizes(n, m, d, POT_PREC_FP32) || !std::isfinite(eps) ||
        eps < 0.f || !finite_pos(tau) || max_iter < 1)
        return POT_ERR_INVALID;
    if (ws_bytes < pot_sinkhorn_divergence_bytes(n, m, d)) return POT_ERR_NOMEM;
    return divergence(X, n, Y, m, d, a, b, 0.f, eps, tau, max_iter, out, ws, ws_bytes,
                      static_cast<hipStream_t>(stream));
}

int pot_sinkhorn_divergence_pcost(const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                                  const float *a, const float *b, float p, float eps, float tau,
                                  int32_t max_iter, double *out, void *ws, size_t ws_bytes,
                                  void *stream) {
    const size_t need = pot_sinkhorn_divergence_pcost_bytes(n, m, d, p);
    if (!X || !Y || !out || !ws || need == 0 || !std::isfinite(eps) || eps < 0.f ||
        !finite_pos(tau) || max_iter < 1)
        return POT_ERR_INVALID;
    if (ws_bytes < need) return POT_ERR_NOMEM;
    return divergence(X, n, Y, m, d, a, b, p, eps, tau, max_iter, out, ws, ws_bytes,
                      static_cast<hipStream_t>(stream));
}

}  // extern "C"

namespace {

// Workspace of pot_sinkhorn_divergence_noalloc: one array per GPU, loaded with
// the library's code object and kept until the process ends.  Host code never
// uses the array's name as an address (on the host it is only a stand-in for
// the symbol): the device address comes from hipGetSymbolAddress, once per
// device, with that device current.
static __device__ __align__(256) unsigned char scratch[POT_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (nullptr on failure).
void *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

int pot_sinkhorn_divergence_noalloc(const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                                    const float *a, const float *b, float eps, float tau,
                                    int32_t max_iter, double *out, void *stream) {
    if (!X || !Y || !out || !valid_sizes(n, m, d, POT_PREC_FP32) || !std::isfinite(eps) ||
        eps < 0.f || !finite_pos(tau) || max_iter < 1)
        return POT_ERR_INVALID;
    const size_t need = pot_sinkhorn_divergence_bytes(n, m, d);
    if (need > (size_t)POT_STATIC_SCRATCH_BYTES) return POT_ERR_NOMEM;
    void *ws = scratch_on_current_device();
    if (!ws) return POT_ERR_DEVICE;
    return divergence(X, n, Y, m, d, a, b, 0.f, eps, tau, max_iter, out, ws, need,
                      static_cast<hipStream_t>(stream), true);
}

int pot_diag_metrics(const pot_clouds *c, const float *f, const float *g, float eps, double *out,
                     void *stream) {
    if (!valid_clouds(c) || !f || !g || !out || !finite_pos(eps) || c->n != c->m)
        return POT_ERR_INVALID;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const Layout L = plan_of(c);
    // the FP64 norm region holds n + m >= 2 diag_blocks(n) doubles
    double *part = at<double>(c, L.n64);
    const int nb = pot::diag_blocks(c->n);
    POT_TRY(pot::launch_diag_sums(c->xk, c->Y, c->n, c->d, f, g, eps, c->cost_p, part, s));
    std::vector<double> h(2 * (size_t)nb);
    POT_TRY(hipMemcpyAsync(h.data(), part, h.size() * 8, hipMemcpyDeviceToHost, s));
    POT_TRY(hipStreamSynchronize(s));
    double tr = 0, slp = 0;
    for (int b = 0; b < nb; ++b) { tr += h[2 * b]; slp += h[2 * b + 1]; }
    const double n = (double)c->n;
    out[0] = tr;
    out[1] = -std::log(n) - slp / n;
    return std::isfinite(tr) ? POT_OK : POT_ERR_NUMERIC;
}

}  // extern "C"
