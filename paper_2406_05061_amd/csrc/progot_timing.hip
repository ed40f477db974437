// Launch timing for the tracing aid of the C ABI (pot_timing_enable /
// pot_timing_read): HIP timing events recorded by the kernel dispatches
// themselves, resolved lazily when read.

#include "progot.h"
#include "progot_internal.h"

#include <mutex>
#include <vector>

namespace {

struct Rec {
    hipEvent_t start, stop;
    int kind;
};

struct Timing {
    std::mutex mu;
    bool on = false;
    int every = 1;                          // time launch 0, every, 2 every, ... of each kind
    int64_t seq[2] = {0, 0};
    std::vector<Rec> live;                  // both recorded, not yet resolved
    std::vector<hipEvent_t> pool;
    double ms[2] = {0.0, 0.0};
    int64_t count[2] = {0, 0};
};

Timing &T() {
    static Timing t;
    return t;
}

hipEvent_t take(Timing &t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold finished records into the totals (caller holds the mutex).
int resolve(Timing &t) {
    int status = POT_OK;
    for (Rec &r : t.live) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) != hipSuccess ||
            hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) {
            status = POT_ERR_DEVICE;
        } else {
            t.ms[r.kind] += ms;
            t.count[r.kind] += 1;
        }
        t.pool.push_back(r.start);
        t.pool.push_back(r.stop);
    }
    t.live.clear();
    return status;
}

}  // namespace

namespace pot {

TimedEvents timing_events(int kind) {
    Timing &t = T();
    std::lock_guard<std::mutex> lk(t.mu);
    if (!t.on || kind < 0 || kind > 1) return {nullptr, nullptr};
    if (t.seq[kind]++ % t.every != 0) return {nullptr, nullptr};
    TimedEvents e{take(t), take(t)};
    if (!e.start || !e.stop) {
        if (e.start) t.pool.push_back(e.start);
        if (e.stop) t.pool.push_back(e.stop);
        return {nullptr, nullptr};
    }
    return e;
}

void timing_commit(int kind, TimedEvents e) {
    if (!e.start) return;
    Timing &t = T();
    std::lock_guard<std::mutex> lk(t.mu);
    // peek: the launch helper reports the launch's own error afterwards
    if (hipPeekAtLastError() == hipSuccess) {
        t.live.push_back(Rec{e.start, e.stop, kind});
    } else {
        t.pool.push_back(e.start);
        t.pool.push_back(e.stop);
    }
}

}  // namespace pot

extern "C" {

int pot_timing_enable(int every) {
    if (every < 0) return POT_ERR_INVALID;
    Timing &t = T();
    std::lock_guard<std::mutex> lk(t.mu);
    int st = resolve(t);
    if (every) {
        t.ms[0] = t.ms[1] = 0.0;
        t.count[0] = t.count[1] = 0;
        t.seq[0] = t.seq[1] = 0;
        t.every = every;
    }
    t.on = every != 0;
    return st;
}

int pot_timing_read(double *lse_ms, int64_t *lse_launches, double *map_ms, int64_t *map_launches) {
    Timing &t = T();
    std::lock_guard<std::mutex> lk(t.mu);
    const int st = resolve(t);
    if (lse_ms) *lse_ms = t.ms[0];
    if (lse_launches) *lse_launches = t.count[0];
    if (map_ms) *map_ms = t.ms[1];
    if (map_launches) *map_launches = t.count[1];
    return st;
}

}  // extern "C"
