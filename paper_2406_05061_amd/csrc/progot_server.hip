// Serving form: continuous batching of ProgOT solves of uneven sizes on one
// GPU.
//
// Requests are admitted while a slot and room in the caller's device arena
// are free (first-fit by HBM footprint, the workspace of one solve).  A tick
// advances every active request by up to kMaxSub Sinkhorn iterations: each
// sub-step runs all f-updates in one grouped, persistent launch per padded
// dimension (a grid of resident workgroups walking the work list), then all
// g-updates; the stop rule runs on the device, and one read-back of every
// request's control word ends the tick.  The requests whose solve ended then
// take their maps (McCann steps and final maps) in one grouped launch per
// padded dimension and move to the next ProgOT step (or finish); new
// requests join at the next tick.  Each request runs the same device bodies
// with the same splits and the same host arithmetic as pot_progot_solve, so
// its result is bit-identical to a solve on its own.

#include "progot.h"
#include "progot_host.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

using namespace pot::host;

namespace {

// First-fit allocator over [0, size) (offsets and sizes multiples of 256).
class FirstFit {
  public:
    void init(size_t size) { free_.assign(1, {0, size}); }
    bool alloc(size_t bytes, size_t *off) {
        for (size_t k = 0; k < free_.size(); ++k) {
            if (free_[k].second >= bytes) {
                *off = free_[k].first;
                free_[k].first += bytes;
                free_[k].second -= bytes;
                if (free_[k].second == 0) free_.erase(free_.begin() + k);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, size_t(0)));
        it = free_.insert(it, {off, bytes});
        // merge with the right neighbour, then the left one
        if (it + 1 != free_.end() && it->first + it->second == (it + 1)->first) {
            it->second += (it + 1)->second;
            free_.erase(it + 1);
        }
        if (it != free_.begin() && (it - 1)->first + (it - 1)->second == it->first) {
            (it - 1)->second += it->second;
            free_.erase(it);
        }
    }

  private:
    std::vector<std::pair<size_t, size_t>> free_;  // (offset, bytes), sorted
};

enum { ST_PREP = 0, ST_SOLVE = 1 };

struct Req {
    int64_t id = 0;
    int state = ST_PREP;
    int slot = 0;
    pot_clouds c{};
    Layout L{};
    size_t off = 0, bytes = 0;
    pot_progot_params p{};
    double eps_explicit[POT_MAX_K];
    float alpha[POT_MAX_K];
    int k = 0, t = 0;
    float eps = 0.f, tau = 0.f, gamma = 1.f;
    const float *g_init = nullptr;
    float *f_out = nullptr, *G = nullptr, *TX = nullptr;
    pot_progot_info info{};
    double t0 = 0.0;
    int status = POT_OK;
    float *fb[2] = {nullptr, nullptr}, *gb[2] = {nullptr, nullptr};
};

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

// A tick gives each request up to kMaxSub iterations: about as many as fit in
// one iteration of the largest active request, and the oldest request at
// least the others' total (small problems would
// otherwise wait on large ones for every single iteration).
constexpr int kMaxSub = 16;

size_t jobs_bytes(int max_active) {
    return a256(sizeof(pot::LseJob) * 2 * (size_t)max_active * kMaxSub);
}
size_t ctl_bytes(int max_active) { return a256(sizeof(int) * 2 * (size_t)max_active); }
// at most one map per request and tick (its McCann step or its final map)
size_t maps_bytes(int max_active) { return a256(sizeof(pot::MapJob) * (size_t)max_active); }

}  // namespace

struct pot_server {
    char *arena = nullptr;
    size_t arena_bytes = 0;
    size_t base = 0;  // first byte of the request region
    hipStream_t s = nullptr;
    int max_active = 0;
    FirstFit fit;
    pot::LseJob *jobs_dev = nullptr;   // in the arena: kMaxSub x (f, g) x max_active
    int *ctl_dev = nullptr;            // in the arena: per slot {stop iterate, err bits}
    pot::MapJob *maps_dev = nullptr;   // in the arena: the tick's grouped maps
    pot::LseJob *jobs_host = nullptr;  // pinned mirror of jobs_dev
    pot::MapJob *maps_host = nullptr;  // pinned mirror of maps_dev
    int *ctl_host = nullptr;           // pinned
    double *mom_host = nullptr;        // pinned, max_active x moments_len(POT_MAX_D)
    std::vector<int> free_slots;
    std::vector<Req *> active;
    std::map<int64_t, Req *> finished;
    int64_t next_id = 1;
};

namespace {

double *moments_slot(pot_server *S, int slot) { return S->mom_host + (size_t)slot * moments_len(POT_MAX_D); }

void release(pot_server *S, Req *r) {
    S->fit.release(r->off, r->bytes);
    S->free_slots.push_back(r->slot);
}

// Move request r to its ProgOT step's Sinkhorn loop (its moments are on the host).
int start_step(pot_server *S, Req *r, const double *mom) {
    int st = finish_moments(&r->c, mom);
    if (st != POT_OK) return st;
    st = step_values(&r->p, r->alpha, r->k, r->c.mean_cost, &r->eps, &r->tau, &r->gamma);
    if (st != POT_OK) return st;
    r->g_init = r->k == 0 ? nullptr : r->G + (size_t)(r->k - 1) * r->c.m;
    r->t = 0;
    r->state = ST_SOLVE;
    POT_TRY(hipMemsetAsync(S->ctl_dev + 2 * r->slot, 0, 2 * sizeof(int), S->s));
    return POT_OK;
}

// Iterate s of step k met its tau (or hit max_iter): store g^(k) and, for the
// last step, f; then describe the map this step ends with -- the McCann step
// of the source in place (next step, *moving) or the final map into TX --
// in *mj (*has_map), for the tick's grouped map launch.  *done when the
// request finishes with this step.
int finish_step(pot_server *S, Req *r, int s_it, float err, bool converged, bool *done, bool *moving,
                pot::MapJob *mj, bool *has_map) {
    pot_clouds *c = &r->c;
    const int64_t m = c->m, n = c->n;
    const int k = r->k;
    r->info.iters[k] = s_it;
    r->info.err[k] = err;
    r->info.eps[k] = r->eps;
    r->info.alpha[k] = r->alpha[k];
    if (!converged) r->info.converged = 0;
    float *Gk = r->G + (size_t)k * m;
    POT_TRY(hipMemcpyAsync(Gk, r->gb[s_it & 1], m * sizeof(float), hipMemcpyDeviceToDevice, S->s));
    // the arguments run_map would pass for this map
    pot::MapArgs a{};
    a.Xq = c->xk; a.nq = n; a.Y = c->Y; a.m = m; a.ysq = c->y_sqn; a.g = Gk; a.eps = r->eps;
    a.d = c->d; a.precision = POT_PREC_FP32;
    if (k + 1 < r->p.K) {
        a.alpha = r->alpha[k]; a.Xout = c->xk; a.out_sqn = c->x_sqn;
        *mj = pot::map_job(a);
        *has_map = true;
        *moving = true;
        *done = false;
    } else {
        POT_TRY(hipMemcpyAsync(r->f_out, r->fb[s_it & 1], n * sizeof(float), hipMemcpyDeviceToDevice,
                               S->s));
        *has_map = r->TX != nullptr;
        if (*has_map) {
            a.alpha = 1.f; a.Xout = r->TX; a.out_sqn = nullptr;
            *mj = pot::map_job(a);
        }
        *moving = false;
        *done = true;
    }
    return POT_OK;
}

}  // namespace

extern "C" {

size_t pot_server_arena_overhead(int32_t max_active) {
    if (max_active < 1 || max_active > POT_SERVER_MAX_ACTIVE) return 0;
    return jobs_bytes(max_active) + ctl_bytes(max_active) + maps_bytes(max_active);
}

size_t pot_server_request_bytes(int64_t n, int64_t m, int32_t d) {
    if (!valid_sizes(n, m, d, POT_PREC_FP32)) return 0;
    return a256(plan(n, m, d, POT_PREC_FP32).total);
}

int pot_server_create(pot_server **out, void *arena, size_t arena_bytes, int32_t max_active,
                      void *stream) {
    if (!out || !arena || max_active < 1 || max_active > POT_SERVER_MAX_ACTIVE) return POT_ERR_INVALID;
    const size_t over = pot_server_arena_overhead(max_active);
    if (arena_bytes <= over) return POT_ERR_NOMEM;
    pot_server *S = new (std::nothrow) pot_server();
    if (!S) return POT_ERR_NOMEM;
    S->arena = static_cast<char *>(arena);
    S->arena_bytes = arena_bytes;
    S->s = static_cast<hipStream_t>(stream);
    S->max_active = max_active;
    S->jobs_dev = reinterpret_cast<pot::LseJob *>(S->arena);
    S->ctl_dev = reinterpret_cast<int *>(S->arena + jobs_bytes(max_active));
    S->maps_dev = reinterpret_cast<pot::MapJob *>(S->arena + jobs_bytes(max_active) + ctl_bytes(max_active));
    S->base = over;
    S->fit.init((arena_bytes - over) & ~size_t(255));
    if (hipHostMalloc(reinterpret_cast<void **>(&S->jobs_host), jobs_bytes(max_active),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&S->ctl_host), ctl_bytes(max_active),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&S->maps_host), maps_bytes(max_active),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&S->mom_host),
                      sizeof(double) * moments_len(POT_MAX_D) * max_active, hipHostMallocDefault) != hipSuccess) {
        pot_server_destroy(S);
        return POT_ERR_DEVICE;
    }
    for (int k = max_active - 1; k >= 0; --k) S->free_slots.push_back(k);
    *out = S;
    return POT_OK;
}

int pot_server_submit(pot_server *S, const float *X, int64_t n, const float *Y, int64_t m, int32_t d,
                      const pot_progot_params *p, float *f, float *G, float *TX, int64_t *rid) {
    if (!S || !X || !Y || !f || !G || !rid || !valid_params(p) || !valid_sizes(n, m, d, POT_PREC_FP32))
        return POT_ERR_INVALID;
    const size_t bytes = pot_server_request_bytes(n, m, d);
    if (bytes > S->arena_bytes - S->base) return POT_ERR_NOMEM;   // can never fit
    if (S->free_slots.empty()) return POT_BUSY;
    size_t off = 0;
    if (!S->fit.alloc(bytes, &off)) return POT_BUSY;
    Req *r = new (std::nothrow) Req();
    if (!r) {
        S->fit.release(off, bytes);
        return POT_ERR_NOMEM;
    }
    r->id = S->next_id++;
    r->slot = S->free_slots.back();
    S->free_slots.pop_back();
    r->off = off;
    r->bytes = bytes;
    r->p = *p;
    if (p->eps_mode == 1) {
        std::copy(p->eps_explicit, p->eps_explicit + p->K, r->eps_explicit);
        r->p.eps_explicit = r->eps_explicit;
    } else {
        r->p.eps_explicit = nullptr;
    }
    alpha_schedule(p->K, p->alpha_sched, r->alpha);
    r->f_out = f; r->G = G; r->TX = TX;
    r->info.K = p->K;
    r->info.converged = 1;
    r->t0 = now_s();
    r->L = plan(n, m, d, POT_PREC_FP32);
    bind_clouds(&r->c, X, n, Y, m, d, nullptr, nullptr, POT_PREC_FP32, S->arena + S->base + off, bytes,
                r->L);
    r->fb[0] = at<float>(&r->c, r->L.f0); r->fb[1] = at<float>(&r->c, r->L.f1);
    r->gb[0] = at<float>(&r->c, r->L.g0); r->gb[1] = at<float>(&r->c, r->L.g1);
    const int st = enqueue_prepare(&r->c, r->L, moments_slot(S, r->slot), S->s);
    if (st != POT_OK) {
        release(S, r);
        delete r;
        return st;
    }
    r->state = ST_PREP;
    S->active.push_back(r);
    *rid = r->id;
    return POT_OK;
}

int pot_server_step(pot_server *S, int32_t *n_active, int32_t *n_finished) {
    if (!S) return POT_ERR_INVALID;
    std::vector<Req *> solving;
    for (Req *r : S->active)
        if (r->state == ST_SOLVE) solving.push_back(r);
    // group by padded dimension (one grouped launch per class and sub-step)
    std::stable_sort(solving.begin(), solving.end(), [](const Req *a, const Req *b) {
        return pot::padded_dim_f32(a->c.d) < pot::padded_dim_f32(b->c.d);
    });
    const int ns = (int)solving.size();
    // iterations per request this tick
    double cmax = 0.0;
    for (Req *r : solving) cmax = std::max(cmax, (double)r->c.n * r->c.m * r->c.d);
    std::vector<int> q(ns);
    int Q = 0;
    for (int i = 0; i < ns; ++i) {
        const Req *r = solving[i];
        const double ratio = cmax / ((double)r->c.n * r->c.m * r->c.d);
        q[i] = (int)std::min<double>(kMaxSub, std::max(1.0, std::floor(ratio)));
        Q = std::max(Q, q[i]);
    }
    // The oldest request also gets at least as much work as all the others
    // together (up to kMaxSub iterations), so it advances at half speed or
    // better however many requests join; without this, processor sharing
    // slows a large request down by the number of comparable ones active,
    // which is what sets the latency tail.
    int head = -1;
    for (int i = 0; i < ns; ++i)
        if (head < 0 || solving[i]->id < solving[head]->id) head = i;
    if (ns > 1) {
        auto work = [&](int i) { return (double)solving[i]->c.n * solving[i]->c.m * solving[i]->c.d; };
        double others = 0.0;
        for (int i = 0; i < ns; ++i)
            if (i != head) others += q[i] * work(i);
        const double need = std::floor(others / work(head));
        q[head] = (int)std::min<double>(kMaxSub, std::max<double>(q[head], need));
        Q = std::max(Q, q[head]);
    }
    // Every sub-step's job tables go into the pinned mirror back to back (f
    // then g per sub-step, each in runs of one dimension class), planned on
    // the host, uploaded in one copy, then launched in order.
    const int A = S->max_active;
    struct Group {
        int off, n;
        pot::GroupPlan plan;
    };
    std::vector<Group> groups;
    int used = 0;   // entries of the mirror written this tick (<= kMaxSub x 2 x A)
    for (int sub = 0; sub < Q; ++sub) {
        std::vector<int> idx;   // requests iterating in this sub-step, by dimension class
        for (int i = 0; i < ns; ++i)
            if (sub < q[i]) idx.push_back(i);
        const int nj = (int)idx.size();
        pot::LseJob *fj = S->jobs_host + used, *gj = fj + nj;
        for (int k = 0; k < nj; ++k) {
            Req *r = solving[idx[k]];
            const int it = r->t + sub + 1;   // iteration run by this sub-step
            pot::LseJob f = f_job(&r->c, r->L, r->eps);
            f.vpot = it == 1 ? r->g_init : r->gb[(it - 1) & 1];
            f.gamma = it == 1 ? r->gamma : 1.f;
            f.pot_old = it == 1 ? nullptr : r->fb[(it - 1) & 1];
            f.pot_out = r->fb[it & 1];
            f.ctl = S->ctl_dev + 2 * r->slot;
            f.iter = it - 1;
            f.max_iter = r->p.max_iter;
            f.tau = r->tau;
            pot::LseJob g = g_job(&r->c, r->L, r->eps);
            g.vpot = r->fb[it & 1];
            g.pot_out = r->gb[it & 1];
            g.ctl = f.ctl;
            fj[k] = f;
            gj[k] = g;
        }
        for (int pass = 0; pass < 2; ++pass) {
            const int base = used + pass * nj;
            int i = 0;
            while (i < nj) {
                int j = i;
                const int D = pot::padded_dim_f32(solving[idx[i]]->c.d);
                while (j < nj && pot::padded_dim_f32(solving[idx[j]]->c.d) == D) ++j;
                Group grp{base + i, j - i, {}};
                POT_TRY(pot::plan_lse_update_group(S->jobs_host + grp.off, grp.n, &grp.plan));
                groups.push_back(grp);
                i = j;
            }
        }
        used += 2 * nj;
    }
    if (used > 0)
        POT_TRY(hipMemcpyAsync(S->jobs_dev, S->jobs_host, sizeof(pot::LseJob) * used, hipMemcpyHostToDevice,
                               S->s));
    for (const Group &grp : groups)
        POT_TRY(pot::enqueue_lse_update_group(S->jobs_dev + grp.off, grp.n, grp.plan, nullptr, S->s));
    POT_TRY(hipMemcpyAsync(S->ctl_host, S->ctl_dev, sizeof(int) * 2 * A, hipMemcpyDeviceToHost, S->s));
    POT_TRY(hipStreamSynchronize(S->s));

    int status = POT_OK;
    std::vector<Req *> done_now, keep, moving;
    int nmap = 0;   // map jobs of this tick, in the pinned mirror
    for (Req *r : S->active) {
        bool done = false;
        int st = POT_OK;
        if (r->state == ST_PREP) {
            // its prepare / move kernels and moments copy completed at the sync
            st = start_step(S, r, moments_slot(S, r->slot));
        } else {
            const int *ctl = S->ctl_host + 2 * r->slot;
            if (ctl[0] != 0) {
                float err;
                std::memcpy(&err, &ctl[1], sizeof(float));
                if (!std::isfinite(err)) {
                    st = POT_ERR_NUMERIC;
                } else {
                    const bool conv = r->tau > 0.f ? err <= r->tau : true;
                    bool mv = false, has_map = false;
                    st = finish_step(S, r, ctl[0], err, conv, &done, &mv, S->maps_host + nmap, &has_map);
                    if (st == POT_OK && has_map) ++nmap;
                    if (st == POT_OK && mv) moving.push_back(r);
                }
            } else {
                const auto pos = std::find(solving.begin(), solving.end(), r) - solving.begin();
                r->t += q[pos];
            }
        }
        if (st != POT_OK) {
            // the failure belongs to this request: it finishes with its
            // status (reported by pot_server_poll) and the others go on; only
            // a failing HIP call is the whole server's error
            r->status = st;
            done = true;
            if (st == POT_ERR_DEVICE) status = st;
        }
        (done ? done_now : keep).push_back(r);
    }
    // The maps every step that ended in this tick finishes with (McCann steps
    // and final maps): one grouped launch per padded dimension, all tables in
    // one upload; then the moved sources' moments (the maps wrote their norms).
    if (nmap > 0) {
        pot::MapJob *mj = S->maps_host;
        std::stable_sort(mj, mj + nmap, [](const pot::MapJob &a, const pot::MapJob &b) {
            return pot::padded_dim_f32(a.d) < pot::padded_dim_f32(b.d);
        });
        std::vector<std::pair<int, int>> runs;   // (offset, count) per dimension class
        std::vector<pot::MapGroupPlan> plans;
        for (int i = 0; i < nmap;) {
            int j = i;
            while (j < nmap && pot::padded_dim_f32(mj[j].d) == pot::padded_dim_f32(mj[i].d)) ++j;
            pot::MapGroupPlan gp;
            POT_TRY(pot::plan_map_group(mj + i, j - i, &gp));
            runs.push_back({i, j - i});
            plans.push_back(gp);
            i = j;
        }
        POT_TRY(hipMemcpyAsync(S->maps_dev, mj, sizeof(pot::MapJob) * nmap, hipMemcpyHostToDevice, S->s));
        for (size_t g = 0; g < runs.size(); ++g)
            POT_TRY(pot::enqueue_map_group(S->maps_dev + runs[g].first, runs[g].second, plans[g], S->s));
    }
    for (Req *r : moving) {
        // fails only when a HIP call does: the whole server's error
        const int st = enqueue_moments(&r->c, r->L, moments_slot(S, r->slot), S->s, true);
        if (st != POT_OK) return st;
        r->k += 1;
        r->state = ST_PREP;
    }
    // (the map tables' upload is complete by the next tick's synchronisation,
    // before the mirror is written again)
    if (!done_now.empty()) {
        POT_TRY(hipStreamSynchronize(S->s));   // final copies and maps are in place
        const double now = now_s();
        for (Req *r : done_now) {
            r->info.seconds = now - r->t0;
            if (r->status == POT_OK && !r->info.converged) r->status = POT_WARN_NOT_CONVERGED;
            release(S, r);
            S->finished[r->id] = r;
        }
    }
    S->active.swap(keep);
    if (n_active) *n_active = (int32_t)S->active.size();
    if (n_finished) *n_finished = (int32_t)done_now.size();
    return status < 0 ? status : POT_OK;
}

int pot_server_poll(pot_server *S, int64_t rid, pot_progot_info *info) {
    if (!S) return POT_ERR_INVALID;
    auto it = S->finished.find(rid);
    if (it == S->finished.end()) {
        for (const Req *r : S->active)
            if (r->id == rid) return POT_BUSY;
        return POT_ERR_INVALID;
    }
    Req *r = it->second;
    if (info) *info = r->info;
    const int st = r->status;
    S->finished.erase(it);
    delete r;
    return st;
}

int pot_server_destroy(pot_server *S) {
    if (!S) return POT_ERR_INVALID;
    (void)hipStreamSynchronize(S->s);
    for (Req *r : S->active) delete r;
    for (auto &kv : S->finished) delete kv.second;
    if (S->jobs_host) (void)hipHostFree(S->jobs_host);
    if (S->ctl_host) (void)hipHostFree(S->ctl_host);
    if (S->maps_host) (void)hipHostFree(S->maps_host);
    if (S->mom_host) (void)hipHostFree(S->mom_host);
    delete S;
    return POT_OK;
}

}  // extern "C"
