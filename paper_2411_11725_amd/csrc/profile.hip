// Per-kernel timing with HIP events (measurement only; off by default).
#include <vector>

#include "nm_internal.h"

namespace nm {

// timing-only events: no system-scope fence (cache write-back) at record time,
// which would otherwise inflate and perturb the kernels being measured
constexpr unsigned kProfEventFlags = hipEventDisableSystemFence;

struct ProfState {
    std::vector<hipEvent_t> pool;                 // free events
    std::vector<int> slot;                        // pending launches
    std::vector<hipEvent_t> start, stop;
    double ms[NM_PROF_SLOTS] = {};
    long long count[NM_PROF_SLOTS] = {};
};

static hipEvent_t take(ProfState *p) {
    if (p->pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, kProfEventFlags) != hipSuccess) return nullptr;
        return e;
    }
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
}

void prof_pair(nm_mesh *m, int s, hipEvent_t *start, hipEvent_t *stop) {
    ProfState *p = m->prof;
    hipEvent_t a = take(p);
    hipEvent_t b = a ? take(p) : nullptr;
    if (!a || !b) {
        if (a) p->pool.push_back(a);
        *start = *stop = nullptr;
        return;
    }
    p->slot.push_back(s);
    p->start.push_back(a);
    p->stop.push_back(b);
    *start = a;
    *stop = b;
}

static void drain(ProfState *p) {
    for (size_t i = 0; i < p->slot.size(); ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->start[i], p->stop[i]) == hipSuccess) {
            p->ms[p->slot[i]] += ms;
            p->count[p->slot[i]] += 1;
        }
        p->pool.push_back(p->start[i]);
        p->pool.push_back(p->stop[i]);
    }
    p->slot.clear();
    p->start.clear();
    p->stop.clear();
}

void prof_free(nm_mesh *m) {
    if (!m->prof) return;
    (void)hipStreamSynchronize(m->stream);
    drain(m->prof);
    for (hipEvent_t e : m->prof->pool) (void)hipEventDestroy(e);
    delete m->prof;
    m->prof = nullptr;
}

}  // namespace nm

using namespace nm;

extern "C" nm_status nm_profile_enable(nm_mesh *m, int on) {
    if (!m) {
        set_error("nm_profile_enable: NULL mesh");
        return NM_EINVAL;
    }
    if (!on) {
        prof_free(m);
        return NM_OK;
    }
    prof_free(m);
    m->prof = new ProfState();
    for (int i = 0; i < 4096; ++i) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, kProfEventFlags) != hipSuccess) break;
        m->prof->pool.push_back(e);
    }
    return NM_OK;
}

extern "C" nm_status nm_profile_read(nm_mesh *m, double ms[NM_PROF_SLOTS], long long counts[NM_PROF_SLOTS]) {
    if (!m || !ms || !counts) {
        set_error("nm_profile_read: NULL argument");
        return NM_EINVAL;
    }
    for (int s = 0; s < NM_PROF_SLOTS; ++s) {
        ms[s] = 0.0;
        counts[s] = 0;
    }
    if (!m->prof) return NM_OK;
    if (hipStreamSynchronize(m->stream) != hipSuccess) {
        set_error("nm_profile_read: stream synchronisation failed");
        return NM_EHIP;
    }
    drain(m->prof);
    for (int s = 0; s < NM_PROF_SLOTS; ++s) {
        ms[s] = m->prof->ms[s];
        counts[s] = m->prof->count[s];
    }
    return NM_OK;
}
