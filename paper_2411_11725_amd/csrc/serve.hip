// Continuous-batching server for independent LLG solves of uneven size.
//
// Requests (host memory, copied at submission) wait in a FIFO queue.  A
// scheduler thread admits them while the device memory of the admitted
// solves (plus the transient tensor set-up of the one being admitted) stays
// within the budget and fewer than max_active run.  Every admitted solve keeps
// its state resident on the device and joins a batch group: solves of one
// shape class (equal padded FFT lengths, node-kernel window and terms) share
// the kernel instantiations, and a group's captured graph advances all of its
// members together, one launch per pass and stage for the whole group.  The
// members' descriptors (buffers, sizes, controller) live in device memory and
// each member keeps its own controller (t, dt, accept), so members finish
// independently; finished solves leave and waiting requests join between
// replays, and the graph is captured once per group, not per member.  Groups
// of different classes replay concurrently on a pool of streams.
//
// A group's batch shape (the column-tile widths of its register-FFT passes
// and its slot count) is chosen per class by timing the batched stage
// kernels on the class's first member, cached per class and device.  Every
// member runs the single-mesh kernels' code on its own buffers, so its
// result does not depend on what else is in the group (nor on the widths,
// which change only how columns are grouped into blocks).
// Device memory of the solves comes from a pool (pool.hip): a finished solve
// gives its buffers back without hipFree, which would wait for the device.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "nm_internal.h"

using namespace nm;

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

int pad_len(int n) {
    if (n <= 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return p;
}

struct Group;

struct Solve {
    uint64_t ticket = 0;
    nm_solve_request req{};
    std::vector<float> Ms, A, alpha, m0;
    // optional cell arrays (empty: absent), in the order staged on the device
    std::vector<float> opt[6];   // Ku, easy, h_cell, D, Kc, cubic
    size_t footprint = 0, setup = 0;
    long long nn = 0, nc = 0;
    nm_mesh *mesh = nullptr;
    float *m_dev = nullptr;
    float *par_dev = nullptr;
    Group *group = nullptr;
    int slot = -1;
    Ctrl *own_ctrl = nullptr;   // the mesh's own controller while it uses the group's
    nm_solve_result res{};
    std::vector<float> m_out;
    // retirement: the final state is copied into pinned staging on the
    // retire stream; the solve is finished once ev has completed
    float *pin = nullptr;
    size_t pin_bytes = 0;
    hipEvent_t ev = nullptr;
    int status = NM_OK;
};

// optional cell arrays of a request: pointer and floats per cell
struct OptArray {
    const float *nm_solve_request::*ptr;
    int per_cell;
};
constexpr OptArray kOpt[6] = {{&nm_solve_request::Ku, 1},     {&nm_solve_request::easy, 3},
                              {&nm_solve_request::h_cell, 3}, {&nm_solve_request::D, 1},
                              {&nm_solve_request::Kc, 1},     {&nm_solve_request::cubic, 6}};

// class key: padded lengths, terms and the node kernel's term instantiation
// (which extra terms the mesh carries).  The node kernel's LDS window is sized
// for the longest rows of the class; a longer window holds the same values
// at the same places, so a member's result does not depend on it.
using ClassKey = std::tuple<int, int, int, unsigned, int>;

ClassKey class_of(const nm_solve_request &r, const nm_mesh *m) {
    return ClassKey{pad_len(r.n[0]), pad_len(r.n[1]), pad_len(r.n[2]), r.terms, node_xt(m, r.terms)};
}

enum SlotState { kFree = 0, kJoining = 1, kRunning = 2 };

struct Group {
    ClassKey key;
    BatchClass bc{};
    int cap = 0;
    hipStream_t stream = nullptr;
    BatchSlot *slots_dev = nullptr;   // cap descriptors read by the graph
    BatchSlot *slots_pin = nullptr;   // pinned staging of the descriptors
    std::vector<BatchSlot> next;      // descriptors for the next replay
    Ctrl *ctrl_dev = nullptr;         // cap controllers
    Ctrl *ctrl_pin = nullptr;         // pinned read-back of the controllers
    std::vector<Solve *> member;
    std::vector<int> state;
    // graphs over the first 1, 2, 4, ... slots: a replay covers the lowest
    // power of two of slots that holds every member (new members take the
    // lowest free slot), so a group that is far from full does not dispatch
    // the blocks of its empty slots
    hipGraphExec_t gexec[5] = {};
    hipEvent_t ev = nullptr;          // end of the last replay and read-back
    int sidx = 0;                     // stream of the replay in flight
    bool inflight = false, dirty = false, wait_admit = false;
};

}  // namespace

struct nm_server {
    nm_server_desc desc{};
    size_t budget = 0, used = 0;
    std::vector<hipStream_t> streams;
    std::vector<int> load;            // replays in flight per stream
    hipStream_t admit_stream = nullptr;
    hipStream_t retire_stream = nullptr;   // result read-back of finished solves
    std::vector<Solve *> retiring;
    std::multimap<size_t, float *> pinned;   // free pinned staging buffers by size
    hipEvent_t admit_ev = nullptr;    // end of the last admission set-up
    int device = 0;
    DevPool *pool = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Solve *> pending;
    int n_active = 0;
    std::vector<Group *> groups;
    std::map<uint64_t, Solve *> done;
    std::map<uint64_t, int> known;  // ticket -> 0 pending / 1 active / 2 done
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
};

namespace {

// batch shape per class and device, chosen by timing (see tune_shape)
struct Shape {
    int cap, tune_y, tune_z;
};
std::mutex g_cap_mu;
std::map<std::tuple<ClassKey, int>, Shape> g_cap;
constexpr int kMaxCap = 16;

size_t solve_footprint(const nm_solve_request &r) {
    nm_mesh_desc d{};
    for (int k = 0; k < 3; ++k) {
        d.n[k] = r.n[k];
        d.h[k] = r.h[k];
    }
    d.gamma = r.gamma;
    const size_t base = nm_mesh_footprint_bytes(&d, NM_DP45);
    if (base == 0) return 0;
    const size_t nn = (size_t)(r.n[0] + 1) * (r.n[1] + 1) * (r.n[2] + 1);
    const size_t nc = (size_t)r.n[0] * r.n[1] * r.n[2];
    size_t staged = 3;   // Ms, A, alpha
    for (const OptArray &o : kOpt)
        if (r.*(o.ptr)) staged += (size_t)o.per_cell;
    return base + sizeof(float) * (3 * nn + staged * nc);   // state + staged parameters
}

// device bytes the tensor set-up of a request takes while it runs (float64
// temporaries, given back to the pool at its end)
size_t solve_setup(const nm_solve_request &r) {
    return kspace_scratch_bytes(r.n[0], r.n[1], r.n[2], pad_len(r.n[0]), pad_len(r.n[1]), pad_len(r.n[2]));
}

// give back the resources of a solve whose stream work has completed
void release(Solve *s, DevPool *pool) {
    if (s->mesh && s->own_ctrl) s->mesh->ctrl = s->own_ctrl;
    if (s->mesh) mesh_release(s->mesh);
    dev_free(s->m_dev, pool);
    dev_free(s->par_dev, pool);
    s->mesh = nullptr;
    s->m_dev = s->par_dev = nullptr;
}

void finish(nm_server *S, Solve *s, int status, bool counted) {
    release(s, S->pool);
    s->res.status = status;
    s->res.t_done = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    if (counted) {
        S->used -= s->footprint;
        S->n_active -= 1;
    }
    S->done[s->ticket] = s;
    S->known[s->ticket] = 2;
    S->cv_done.notify_all();
}

void group_destroy(Group *g, DevPool *pool) {
    for (hipGraphExec_t x : g->gexec)
        if (x) (void)hipGraphExecDestroy(x);
    if (g->ev) (void)hipEventDestroy(g->ev);
    dev_free(g->slots_dev, pool);
    dev_free(g->ctrl_dev, pool);
    if (g->slots_pin) (void)hipHostFree(g->slots_pin);
    if (g->ctrl_pin) (void)hipHostFree(g->ctrl_pin);
    delete g;
}

// one replay's kernels: attempts DP45 attempts of the first `slots` slots
hipError_t enqueue_attempts(const Group *g, int slots, int attempts, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int a = 0; a < attempts && e == hipSuccess; ++a) {
        for (int s = 2; s <= 7 && e == hipSuccess; ++s) {
            if (g->bc.terms & NM_T_DEMAG) e = launch_batch_demag(g->bc, g->slots_dev, slots, s, st);
            if (e == hipSuccess) e = launch_batch_node(g->bc, g->slots_dev, slots, s, st);
        }
        if (e == hipSuccess) e = launch_batch_control(g->slots_dev, slots, st);
        if (e == hipSuccess) e = launch_batch_finish(g->bc, g->slots_dev, slots, st);
    }
    return e;
}

// Batch shape of a class, from the stage-2 kernels (demag passes and the
// node kernel) on slots that all describe the class's first member, timed
// on the group's stream (a warm-up and two timings of 2 launches, the faster
// kept): first the column-tile widths of the y passes and the z convolution
// on one slot (the widest unless another is 5% faster), then the slot count,
// doubled from 1 while the time per slot falls by at least 10% (members of a
// fuller group wait longer for each other; stopping at the first doubling
// that does not pay keeps the timing of large classes, which fill the GPU
// with one slot, to two launches' worth).  The timing runs inside the
// stream of requests, so it is kept short: a class costs a few tens of
// launches once per device.  Stage 2 writes only the first member's stage
// buffers and FFT workspace, which its first real attempt rewrites before
// reading.
Shape tune_shape(nm_server *S, Group *g, const BatchSlot &first) {
    const auto ck = std::make_tuple(g->key, S->device);
    {
        std::lock_guard<std::mutex> lk(g_cap_mu);
        auto it = g_cap.find(ck);
        if (it != g_cap.end()) return it->second;
    }
    for (int i = 0; i < kMaxCap; ++i) g->slots_pin[i] = first;
    hipError_t e = hipMemcpyAsync(g->slots_dev, g->slots_pin, sizeof(BatchSlot) * kMaxCap, hipMemcpyHostToDevice,
                                  g->stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto stage2 = [&](int c) -> hipError_t {
        hipError_t r = hipSuccess;
        if (g->bc.terms & NM_T_DEMAG) r = launch_batch_demag(g->bc, g->slots_dev, c, 2, g->stream);
        if (r == hipSuccess) r = launch_batch_node(g->bc, g->slots_dev, c, 2, g->stream);
        return r;
    };
    auto time_c = [&](int c, float *ms_out) -> hipError_t {
        float best = 1e30f;
        hipError_t r = stage2(c);   // warm-up
        for (int rep = 0; rep < 2 && r == hipSuccess; ++rep) {
            r = hipEventRecord(e0, g->stream);
            for (int q = 0; q < 2 && r == hipSuccess; ++q) r = stage2(c);
            if (r == hipSuccess) r = hipEventRecord(e1, g->stream);
            if (r == hipSuccess) r = hipEventSynchronize(e1);
            float ms = 0.f;
            if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
            best = std::fmin(best, ms);
        }
        *ms_out = best;
        return r;
    };
    auto pick_width = [&](int *w, int nw) {
        float t[3] = {1e30f, 1e30f, 1e30f};
        for (int v = 0; v < nw && e == hipSuccess; ++v) {
            *w = v;
            e = time_c(1, &t[v]);
        }
        int b = 0;
        for (int v = 1; v < nw; ++v)
            if (t[v] < 0.95f * t[b]) b = v;
        *w = b;
    };
    Shape sh{1, 0, 0};
    if ((g->bc.terms & NM_T_DEMAG) && g->bc.P3 > 1) {
        pick_width(&g->bc.tune_y, tile_widths(g->bc.P2));
        pick_width(&g->bc.tune_z, tile_widths(g->bc.P3));
    }
    sh.tune_y = g->bc.tune_y;
    sh.tune_z = g->bc.tune_z;
    float prev = 0.f;
    for (int k = 0; (1 << k) <= kMaxCap && e == hipSuccess; ++k) {
        float t = 0.f;
        e = time_c(1 << k, &t);
        t /= (float)(1 << k);
        if (e != hipSuccess || (k > 0 && t > 0.9f * prev)) break;
        sh.cap = 1 << k;
        prev = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(g_cap_mu);
    g_cap[ck] = sh;
    return sh;
}

// the stream with the fewest replays in flight (lowest index on ties)
int least_loaded(const nm_server *S) {
    int b = 0;
    for (int i = 1; i < (int)S->load.size(); ++i)
        if (S->load[i] < S->load[b]) b = i;
    return b;
}

// pinned staging of at least `bytes`: a free buffer of the server, else a new
// one rounded up to a power of two (kept until the server is destroyed)
float *pinned_get(nm_server *S, size_t bytes, size_t *got) {
    auto it = S->pinned.lower_bound(bytes);
    if (it != S->pinned.end()) {
        float *p = it->second;
        *got = it->first;
        S->pinned.erase(it);
        return p;
    }
    size_t sz = 4096;
    while (sz < bytes) sz <<= 1;
    void *p = nullptr;
    if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
    *got = sz;
    return static_cast<float *>(p);
}

// Grid extents of a group: its launches cover the largest rows, layers and
// node ranges of the members its graphs were captured for, and the LDS
// window of their longest rows (a longer window holds the same values at the
// same places, so a member's result depends on neither).
struct Extents {
    int N2 = 0, N3 = 0, NX = 0, NZ = 0;
    int np = 0;
};
void grow(Extents *x, const BatchSlot &d) {
    x->N2 = std::max(x->N2, d.N2);
    x->N3 = std::max(x->N3, d.N3);
    x->NX = std::max(x->NX, d.N1 + 1);
    x->NZ = std::max(x->NZ, d.NZ);
    x->np = std::max(x->np, d.np);
}
void set_extents(Group *g, const Extents &x) {
    g->bc.gN2 = x.N2;
    g->bc.gN3 = x.N3;
    g->bc.node_blocks = (unsigned)x.np;
    g->bc.nit = window_items(x.NX, x.NZ);
}

// create the group of a class on the first admitted member (its descriptor
// is used to time the batch shapes)
Group *group_create(nm_server *S, const ClassKey &key, const Solve *first, const BatchSlot &desc) {
    Group *g = new Group();
    g->key = key;
    g->bc.P1 = std::get<0>(key);
    g->bc.P2 = std::get<1>(key);
    g->bc.P3 = std::get<2>(key);
    g->bc.terms = std::get<3>(key);
    g->bc.xt = std::get<4>(key);
    g->bc.tune_y = g->bc.tune_z = 0;
    Extents x{};
    grow(&x, desc);
    set_extents(g, x);
    g->sidx = least_loaded(S);
    g->stream = S->streams[g->sidx];
    bool ok = dev_alloc((void **)&g->slots_dev, sizeof(BatchSlot) * kMaxCap, S->pool) == hipSuccess &&
              dev_alloc((void **)&g->ctrl_dev, sizeof(Ctrl) * kMaxCap, S->pool) == hipSuccess &&
              hipHostMalloc((void **)&g->slots_pin, sizeof(BatchSlot) * kMaxCap, hipHostMallocDefault) == hipSuccess &&
              hipHostMalloc((void **)&g->ctrl_pin, sizeof(Ctrl) * kMaxCap, hipHostMallocDefault) == hipSuccess &&
              hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) == hipSuccess;
    // the timing runs after the member's set-up
    ok = ok && hipStreamWaitEvent(g->stream, S->admit_ev, 0) == hipSuccess;
    if (!ok) {
        group_destroy(g, S->pool);
        return nullptr;
    }
    const Shape sh = tune_shape(S, g, desc);
    g->cap = sh.cap;
    g->bc.tune_y = sh.tune_y;
    g->bc.tune_z = sh.tune_z;
    BatchSlot empty{};
    g->next.assign(g->cap, empty);
    g->member.assign(g->cap, nullptr);
    g->state.assign(g->cap, kFree);
    return g;
}

// upload, create the mesh and its tensor, start the integrator (first
// stage, on the admission stream) and place the solve in a group slot
bool admit(nm_server *S, Solve *s) {
    const nm_solve_request &r = s->req;
    s->nc = (long long)r.n[0] * r.n[1] * r.n[2];
    s->nn = (long long)(r.n[0] + 1) * (r.n[1] + 1) * (r.n[2] + 1);
    hipStream_t st = S->admit_stream;
    size_t staged = 3 * (size_t)s->nc;
    for (const std::vector<float> &v : s->opt) staged += v.size();
    if (dev_alloc((void **)&s->par_dev, sizeof(float) * staged, S->pool) != hipSuccess) return false;
    if (dev_alloc((void **)&s->m_dev, sizeof(float) * 3 * s->nn, S->pool) != hipSuccess) return false;
    float *Ms = s->par_dev, *A = s->par_dev + s->nc, *al = s->par_dev + 2 * s->nc;
    const size_t cb = sizeof(float) * s->nc;
    if (hipMemcpyAsync(Ms, s->Ms.data(), cb, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    if (hipMemcpyAsync(A, s->A.data(), cb, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    if (hipMemcpyAsync(al, s->alpha.data(), cb, hipMemcpyHostToDevice, st) != hipSuccess) return false;
    const float *opt_dev[6] = {};
    float *next = s->par_dev + 3 * s->nc;
    for (int i = 0; i < 6; ++i) {
        if (s->opt[i].empty()) continue;
        if (hipMemcpyAsync(next, s->opt[i].data(), sizeof(float) * s->opt[i].size(), hipMemcpyHostToDevice, st) !=
            hipSuccess)
            return false;
        opt_dev[i] = next;
        next += s->opt[i].size();
    }
    if (hipMemcpyAsync(s->m_dev, s->m0.data(), sizeof(float) * 3 * s->nn, hipMemcpyHostToDevice, st) != hipSuccess)
        return false;
    nm_mesh_desc d{};
    for (int k = 0; k < 3; ++k) {
        d.n[k] = r.n[k];
        d.h[k] = r.h[k];
    }
    d.gamma = r.gamma;
    d.stream = st;
    nm_material mat{};
    mat.Ms = Ms;
    mat.A = A;
    mat.alpha = al;
    for (int k = 0; k < 3; ++k) mat.h_uniform[k] = r.h_uniform[k];
    mat.Ku = opt_dev[0];
    mat.easy = opt_dev[1];
    mat.h_cell = opt_dev[2];
    mat.D = opt_dev[3];
    mat.dmi_type = r.dmi_type;
    mat.Kc = opt_dev[4];
    mat.cubic = opt_dev[5];
    if (nm_mesh_create(&d, &mat, &s->mesh) != NM_OK) return false;
    // the tensor without the per-mesh tile tuner: the group's kernels take
    // the widths tuned for the whole class
    if (r.terms & NM_T_DEMAG) {
        if (build_kspace_tensor(s->mesh) != hipSuccess) return false;
        s->mesh->tensor_ready = true;
    }
    nm_integrator in{};
    in.method = NM_DP45;
    in.terms = r.terms;
    in.rtol = r.rtol;
    in.atol = r.atol;
    in.dt_min = 1e-20;
    nm_clock clk{0.0, r.dt0, 0, 0, 0, 0.0};
    int batch = 0;
    if (step_begin(s->mesh, s->m_dev, &clk, &in, r.t_end, 1L << 40, &batch) != NM_OK) return false;
    // its group: one of the class with a free slot, else a new one
    const ClassKey key = class_of(r, s->mesh);
    Group *g = nullptr;
    int slot = -1;
    for (Group *x : S->groups) {
        if (x->key != key) continue;
        for (int i = 0; i < x->cap; ++i)
            if (x->state[i] == kFree) {
                g = x;
                slot = i;
                break;
            }
        if (g) break;
    }
    BatchSlot desc{};
    if (hipEventRecord(S->admit_ev, st) != hipSuccess) return false;
    if (!g) {
        // the controller the timing's stage-2 kernels read: the mesh's own
        batch_slot_fill(s->mesh, r.terms, s->mesh->ctrl, s->m_dev, &desc);
        g = group_create(S, key, s, desc);
        if (!g) return false;
        S->groups.push_back(g);
        slot = 0;
    }
    // the group's controller of the slot starts as the mesh's (after the first stage)
    if (hipMemcpyAsync(g->ctrl_dev + slot, s->mesh->ctrl, sizeof(Ctrl), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return false;
    if (hipEventRecord(S->admit_ev, st) != hipSuccess) return false;
    batch_slot_fill(s->mesh, r.terms, g->ctrl_dev + slot, s->m_dev, &desc);
    // from here on the mesh's own kernels (a group with this member alone
    // replays them) use the group's controller of the slot too, and the
    // class's column-tile widths
    s->own_ctrl = s->mesh->ctrl;
    s->mesh->ctrl = g->ctrl_dev + slot;
    s->mesh->tune_y = g->bc.tune_y;
    s->mesh->tune_z = g->bc.tune_z;
    g->next[slot] = desc;
    g->member[slot] = s;
    g->state[slot] = kJoining;
    g->dirty = true;
    g->wait_admit = true;
    s->group = g;
    s->slot = slot;
    s->res.t_admit = now_s();
    return true;
}

// a finished member leaves its slot at once; its final state is copied to
// pinned staging on the retire stream (after the replay that finished it,
// which has completed), and the solve is finished by retire() once that copy
// has landed, so the scheduler never waits for a copy or for other groups'
// work on a replay stream
void complete(nm_server *S, Group *g, int slot) {
    Solve *s = g->member[slot];
    const Ctrl &C = g->ctrl_pin[slot];
    s->res.t = C.t;
    s->res.accepted = C.accepted;
    s->res.rejected = C.rejected;
    s->res.rhs_evals = C.rhs_evals + 1;   // + the first stage
    s->status = C.status == NM_ENONFINITE ? NM_ENONFINITE : C.status == NM_ESTEPSIZE ? NM_ESTEPSIZE : NM_OK;
    const size_t bytes = sizeof(float) * 3 * s->nn;
    hipError_t e = hipEventCreateWithFlags(&s->ev, hipEventDisableTiming);
    if (e == hipSuccess) {
        s->pin = pinned_get(S, bytes, &s->pin_bytes);
        if (!s->pin) e = hipErrorOutOfMemory;
    }
    if (e == hipSuccess) e = hipMemcpyAsync(s->pin, s->m_dev, bytes, hipMemcpyDeviceToHost, S->retire_stream);
    if (e == hipSuccess) e = hipEventRecord(s->ev, S->retire_stream);
    if (e != hipSuccess) {
        // fall back to a blocking copy so the result is not lost
        (void)hipGetLastError();
        s->m_out.resize(3 * s->nn);
        if (hipMemcpy(s->m_out.data(), s->m_dev, bytes, hipMemcpyDeviceToHost) != hipSuccess) s->status = NM_EHIP;
        if (s->pin) S->pinned.emplace(s->pin_bytes, s->pin);
        s->pin = nullptr;
        if (s->ev) (void)hipEventDestroy(s->ev);
        s->ev = nullptr;
    }
    g->member[slot] = nullptr;
    g->state[slot] = kFree;
    g->next[slot].active = 0;
    g->dirty = true;
    S->retiring.push_back(s);
}

// finish the retiring solves whose read-back has landed; true if any did
bool retire(nm_server *S) {
    bool any = false;
    for (size_t i = 0; i < S->retiring.size();) {
        Solve *s = S->retiring[i];
        if (s->ev) {
            const hipError_t q = hipEventQuery(s->ev);
            if (q == hipErrorNotReady) {
                (void)hipGetLastError();
                ++i;
                continue;
            }
            if (q == hipSuccess) {
                s->m_out.assign(s->pin, s->pin + 3 * s->nn);
            } else {
                s->status = NM_EHIP;
            }
            (void)hipEventDestroy(s->ev);
            s->ev = nullptr;
            S->pinned.emplace(s->pin_bytes, s->pin);
            s->pin = nullptr;
        }
        S->retiring[i] = S->retiring.back();
        S->retiring.pop_back();
        finish(S, s, s->status, true);
        any = true;
    }
    return any;
}

// issue one replay of an idle group: new descriptors, the graph, the
// controllers' read-back
hipError_t issue(nm_server *S, Group *g) {
    hipError_t e = hipSuccess;
    // the group's previous replay has completed, so its next one may go to
    // any stream: the one with the fewest replays in flight
    g->sidx = least_loaded(S);
    g->stream = S->streams[g->sidx];
    if (g->dirty) {
        std::memcpy(g->slots_pin, g->next.data(), sizeof(BatchSlot) * g->cap);
        e = hipMemcpyAsync(g->slots_dev, g->slots_pin, sizeof(BatchSlot) * g->cap, hipMemcpyHostToDevice, g->stream);
        for (int i = 0; i < g->cap; ++i)
            if (g->state[i] == kJoining) g->state[i] = kRunning;
        g->dirty = false;
    }
    if (e == hipSuccess && g->wait_admit) {
        e = hipStreamWaitEvent(g->stream, S->admit_ev, 0);
        g->wait_admit = false;
    }
    // a group with one member replays that member's own single-mesh graph
    // (the kernels nm_llg_step runs, with its exact grids and parameters in
    // the kernel arguments) on the chosen stream; the batched kernels, which
    // first read each slot's descriptor from device memory, only where they
    // serve several members
    int occupied = 0, only = -1;
    for (int i = 0; i < g->cap; ++i)
        if (g->state[i] != kFree) {
            ++occupied;
            only = i;
        }
    if (occupied == 1) {
        Solve *s1 = g->member[only];
        s1->mesh->stream = g->stream;
        const int A = S->desc.attempts_per_launch;
        if (e == hipSuccess) e = step_batch(s1->mesh, s1->m_dev, NM_DP45, g->bc.terms, A, A);
        if (e == hipSuccess)
            e = hipMemcpyAsync(g->ctrl_pin, g->ctrl_dev, sizeof(Ctrl) * g->cap, hipMemcpyDeviceToHost, g->stream);
        if (e == hipSuccess) e = hipEventRecord(g->ev, g->stream);
        if (e == hipSuccess) {
            g->inflight = true;
            S->load[g->sidx] += 1;
        }
        return e;
    }
    // refit the grids to the members: grow when a member exceeds them, shrink
    // when they cover more than 5/4 of the node blocks needed; either way the
    // captured graphs are dropped and recaptured on demand
    {
        Extents x{};
        for (int i = 0; i < g->cap; ++i)
            if (g->state[i] != kFree) grow(&x, g->next[i]);
        const BatchClass &c = g->bc;
        const bool over = x.N2 > c.gN2 || x.N3 > c.gN3 || x.np > (int)c.node_blocks ||
                          window_items(x.NX, x.NZ) != c.nit;
        const bool slack = 4 * (long long)c.node_blocks > 5LL * x.np;
        if (x.np > 0 && (over || slack)) {
            for (hipGraphExec_t &ge : g->gexec) {
                if (ge) (void)hipGraphExecDestroy(ge);
                ge = nullptr;
            }
            set_extents(g, x);
        }
    }
    // the smallest power of two of slots that covers every occupied slot
    int hi = 0;
    for (int i = 0; i < g->cap; ++i)
        if (g->state[i] != kFree) hi = i + 1;
    int k = 0;
    while ((1 << k) < hi) ++k;
    const int slots = std::min(1 << k, g->cap);
    if (e == hipSuccess && !g->gexec[k]) {
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed);
        hipError_t e2 = e == hipSuccess ? enqueue_attempts(g, slots, S->desc.attempts_per_launch, g->stream) : e;
        if (e == hipSuccess) e = hipStreamEndCapture(g->stream, &graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&g->gexec[k], graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e == hipSuccess) e = hipGraphUpload(g->gexec[k], g->stream);
    }
    if (e == hipSuccess) e = hipGraphLaunch(g->gexec[k], g->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(g->ctrl_pin, g->ctrl_dev, sizeof(Ctrl) * g->cap, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipEventRecord(g->ev, g->stream);
    if (e == hipSuccess) {
        g->inflight = true;
        S->load[g->sidx] += 1;
    }
    return e;
}

void fail_group(nm_server *S, Group *g) {
    (void)hipStreamSynchronize(g->stream);
    for (int i = 0; i < g->cap; ++i)
        if (g->member[i]) {
            finish(S, g->member[i], NM_EHIP, true);
            g->member[i] = nullptr;
            g->state[i] = kFree;
            g->next[i].active = 0;
        }
    g->dirty = true;
    g->inflight = false;
}

void run(nm_server *S) {
    (void)hipSetDevice(S->device);
    set_thread_pool(S->pool);
    for (;;) {
        // admission: FIFO, within the memory budget and the active cap
        for (;;) {
            Solve *s = nullptr;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                if (S->stop) return;
                if (S->n_active == 0 && S->pending.empty()) {
                    S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
                    if (S->stop) return;
                }
                if (S->pending.empty() || S->n_active >= S->desc.max_active) break;
                Solve *f = S->pending.front();
                if (S->used + f->footprint + f->setup > S->budget) {
                    if (S->n_active > 0) break;   // wait for memory to free up
                    S->pending.pop_front();        // can never fit
                    lk.unlock();
                    finish(S, f, NM_EBUDGET, false);
                    continue;
                }
                S->pending.pop_front();
                S->used += f->footprint;
                S->n_active += 1;
                S->known[f->ticket] = 1;
                s = f;
            }
            if (!admit(S, s)) {
                (void)hipStreamSynchronize(S->admit_stream);
                if (s->group) {
                    Group *g = s->group;
                    g->member[s->slot] = nullptr;
                    g->state[s->slot] = kFree;
                    g->next[s->slot].active = 0;
                    g->dirty = true;
                }
                finish(S, s, NM_EHIP, true);
            }
        }
        // retire finished members of groups whose replay has ended, then
        // issue a replay for every idle group with running members
        bool progressed = false;
        for (Group *g : S->groups) {
            if (g->inflight) {
                const hipError_t q = hipEventQuery(g->ev);
                if (q == hipErrorNotReady) {
                    (void)hipGetLastError();   // not an error: keep it out of later checks
                    continue;
                }
                g->inflight = false;
                S->load[g->sidx] -= 1;
                progressed = true;
                if (q != hipSuccess) {
                    fail_group(S, g);
                    continue;
                }
                for (int i = 0; i < g->cap; ++i)
                    if (g->state[i] == kRunning && g->ctrl_pin[i].done) complete(S, g, i);
            }
            bool any = false;
            for (int i = 0; i < g->cap; ++i) any = any || g->state[i] != kFree;
            if (!any) continue;
            if (issue(S, g) != hipSuccess) {
                fail_group(S, g);
                continue;
            }
            progressed = true;
        }
        if (retire(S)) progressed = true;
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace

#define NM_REQUIRE(cond, code, msg) \
    do {                            \
        if (!(cond)) {              \
            set_error(msg);         \
            return code;            \
        }                           \
    } while (0)

extern "C" nm_status nm_server_create(const nm_server_desc *desc, nm_server **out) {
    NM_REQUIRE(desc && out, NM_EINVAL, "nm_server_create: NULL argument");
    NM_REQUIRE(desc->max_active >= 1, NM_EINVAL, "nm_server_create: max_active must be >= 1");
    NM_REQUIRE(desc->n_streams >= 1 && desc->n_streams <= 16, NM_EINVAL,
               "nm_server_create: n_streams must be in 1..16");
    NM_REQUIRE(desc->attempts_per_launch >= 1 && desc->attempts_per_launch <= 64, NM_EINVAL,
               "nm_server_create: attempts_per_launch must be in 1..64");
    nm_server *S = new nm_server();
    S->desc = *desc;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        set_error("nm_server_create: no device");
        return NM_EHIP;
    }
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess) freeb = 0;
    S->budget = desc->hbm_budget ? desc->hbm_budget : (size_t)(0.8 * (double)freeb);
    bool ok = true;
    for (int i = 0; i < desc->n_streams + 2 && ok; ++i) {
        hipStream_t st = nullptr;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (!ok) break;
        if (i < desc->n_streams) S->streams.push_back(st);
        else if (i == desc->n_streams) S->admit_stream = st;
        else S->retire_stream = st;
    }
    S->load.assign(S->streams.size(), 0);
    ok = ok && hipEventCreateWithFlags(&S->admit_ev, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
        if (S->admit_stream) (void)hipStreamDestroy(S->admit_stream);
        if (S->retire_stream) (void)hipStreamDestroy(S->retire_stream);
        if (S->admit_ev) (void)hipEventDestroy(S->admit_ev);
        delete S;
        set_error("nm_server_create: stream creation failed");
        return NM_EHIP;
    }
    S->pool = pool_create();
    S->worker = std::thread(run, S);
    *out = S;
    return NM_OK;
}

extern "C" nm_status nm_server_destroy(nm_server *S) {
    if (!S) return NM_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->worker.join();
    for (hipStream_t x : S->streams) (void)hipStreamSynchronize(x);
    (void)hipStreamSynchronize(S->admit_stream);
    (void)hipStreamSynchronize(S->retire_stream);
    for (Solve *s : S->retiring) {
        release(s, S->pool);
        if (s->ev) (void)hipEventDestroy(s->ev);
        delete s;
    }
    for (auto &kv : S->pinned) (void)hipHostFree(kv.second);
    for (Group *g : S->groups) {
        for (Solve *s : g->member)
            if (s) {
                release(s, S->pool);
                delete s;
            }
        group_destroy(g, S->pool);
    }
    for (Solve *s : S->pending) delete s;
    for (auto &kv : S->done) delete kv.second;
    for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
    (void)hipStreamDestroy(S->admit_stream);
    (void)hipStreamDestroy(S->retire_stream);
    (void)hipEventDestroy(S->admit_ev);
    pool_destroy(S->pool);
    delete S;
    return NM_OK;
}

extern "C" nm_status nm_serve_submit(nm_server *S, const nm_solve_request *r, uint64_t *ticket) {
    NM_REQUIRE(S && r && ticket, NM_EINVAL, "nm_serve_submit: NULL argument");
    NM_REQUIRE(r->Ms && r->A && r->alpha && r->m0, NM_EINVAL, "nm_serve_submit: Ms, A, alpha and m0 are required");
    NM_REQUIRE(r->t_end > 0.0 && r->dt0 > 0.0 && r->rtol > 0.0 && r->atol > 0.0, NM_EINVAL,
               "nm_serve_submit: need t_end, dt0, rtol, atol > 0");
    NM_REQUIRE(!(r->terms & ~(unsigned)NM_T_ALL), NM_EINVAL, "nm_serve_submit: unknown term bits");
    NM_REQUIRE(r->n[2] <= 128, NM_EINVAL, "nm_serve_submit: the server takes at most 128 cells along z");
    NM_REQUIRE((r->Ku == nullptr) == (r->easy == nullptr), NM_EINVAL,
               "nm_serve_submit: Ku and easy must be given together");
    NM_REQUIRE((r->Kc == nullptr) == (r->cubic == nullptr), NM_EINVAL,
               "nm_serve_submit: Kc and cubic must be given together");
    NM_REQUIRE(r->dmi_type == NM_DMI_INTERFACIAL || r->dmi_type == NM_DMI_BULK, NM_EINVAL,
               "nm_serve_submit: unknown dmi_type");
    const size_t fp = solve_footprint(*r);
    NM_REQUIRE(fp > 0, NM_EINVAL, "nm_serve_submit: unsupported mesh size");
    Solve *s = new Solve();
    s->req = *r;
    s->footprint = fp;
    s->setup = (r->terms & NM_T_DEMAG) ? solve_setup(*r) : 0;
    const size_t nc = (size_t)r->n[0] * r->n[1] * r->n[2];
    const size_t nn = (size_t)(r->n[0] + 1) * (r->n[1] + 1) * (r->n[2] + 1);
    s->Ms.assign(r->Ms, r->Ms + nc);
    s->A.assign(r->A, r->A + nc);
    s->alpha.assign(r->alpha, r->alpha + nc);
    s->m0.assign(r->m0, r->m0 + 3 * nn);
    s->req.Ms = s->req.A = s->req.alpha = s->req.m0 = nullptr;
    for (int i = 0; i < 6; ++i) {
        const float *src = r->*(kOpt[i].ptr);
        if (src) s->opt[i].assign(src, src + kOpt[i].per_cell * nc);
        s->req.*(kOpt[i].ptr) = nullptr;
    }
    s->res.status = NM_ENOTREADY;
    s->res.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        s->ticket = S->next_ticket++;
        S->known[s->ticket] = 0;
        S->pending.push_back(s);
    }
    S->cv_work.notify_all();
    *ticket = s->ticket;
    return NM_OK;
}

extern "C" nm_status nm_serve_poll(nm_server *S, uint64_t ticket, nm_solve_result *res, float *m_out,
                                   int timeout_ms) {
    NM_REQUIRE(S && res, NM_EINVAL, "nm_serve_poll: NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    if (!S->known.count(ticket)) {
        set_error("nm_serve_poll: unknown ticket");
        return NM_EINVAL;
    }
    auto ready = [&] { return S->done.count(ticket) > 0; };
    if (!ready() && timeout_ms > 0)
        S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (!ready()) {
        res->status = NM_ENOTREADY;
        return NM_ENOTREADY;
    }
    Solve *s = S->done[ticket];
    *res = s->res;
    if (m_out && !s->m_out.empty()) std::memcpy(m_out, s->m_out.data(), sizeof(float) * s->m_out.size());
    S->done.erase(ticket);
    S->known.erase(ticket);
    delete s;
    return NM_OK;
}

extern "C" double nm_server_clock(void) { return now_s(); }
