// Continuous-batching server for independent LLG solves of uneven size.
//
// Requests (host memory, copied at submission) wait in a FIFO queue.  A
// scheduler thread admits them while the device memory of the admitted
// solves stays within the budget and fewer than max_active run; every
// admitted solve keeps its state resident on the device and advances by
// replays of its own captured Dormand-Prince graph (attempts_per_launch
// attempts each) on one stream of a pool, so the work of many solves is in
// flight on the GPU at once.  Solves progress independently: a replay is
// re-issued as soon as the previous one has finished, finished solves leave
// and waiting requests join between replays.  Device memory of the solves
// comes from a pool (pool.hip): a finished solve gives its buffers back
// without hipFree, which would wait for the whole device.  Every solve runs
// the same kernels on its own buffers, so its result does not depend on what
// else is in the mix.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "nm_internal.h"

using namespace nm;

namespace {

double now_s() {
    using clk = std::chrono::steady_clock;
    static const clk::time_point t0 = clk::now();
    return std::chrono::duration<double>(clk::now() - t0).count();
}

struct Solve {
    uint64_t ticket = 0;
    nm_solve_request req{};
    std::vector<float> Ms, A, alpha, m0;
    size_t footprint = 0;
    long long nn = 0, nc = 0;
    nm_mesh *mesh = nullptr;
    float *m_dev = nullptr;
    float *par_dev = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    int batch = 16;
    int next = 16;           // attempts in the next replay (fewer near the end)
    bool inflight = false;
    nm_clock clk{};
    nm_solve_result res{};
    std::vector<float> m_out;
};

}  // namespace

struct nm_server {
    nm_server_desc desc{};
    size_t budget = 0, used = 0;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    int device = 0;
    DevPool *pool = nullptr;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Solve *> pending;
    std::vector<Solve *> active;
    std::map<uint64_t, Solve *> done;
    std::map<uint64_t, int> known;  // ticket -> 0 pending / 1 active / 2 done
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
};

namespace {

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
    return base + sizeof(float) * (3 * nn + 3 * nc);   // state + staged parameters
}

// give back the resources of a solve whose stream work has completed
void release(Solve *s, DevPool *pool) {
    if (s->mesh) mesh_release(s->mesh);
    dev_free(s->m_dev, pool);
    dev_free(s->par_dev, pool);
    if (s->ev) (void)hipEventDestroy(s->ev);
    s->mesh = nullptr;
    s->m_dev = s->par_dev = nullptr;
    s->ev = nullptr;
}

void fail(nm_server *S, Solve *s, int status) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);   // rare path: drain before reuse
    release(s, S->pool);
    s->res.status = status;
    s->res.t_done = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    S->done[s->ticket] = s;
    S->known[s->ticket] = 2;
    S->cv_done.notify_all();
}

// upload, create the mesh and its tensor, start the integrator; on the solve's stream
bool admit(nm_server *S, Solve *s) {
    s->stream = S->streams[S->next_stream++ % S->streams.size()];
    const nm_solve_request &r = s->req;
    s->nc = (long long)r.n[0] * r.n[1] * r.n[2];
    s->nn = (long long)(r.n[0] + 1) * (r.n[1] + 1) * (r.n[2] + 1);
    if (dev_alloc((void **)&s->par_dev, sizeof(float) * 3 * s->nc, S->pool) != hipSuccess) return false;
    if (dev_alloc((void **)&s->m_dev, sizeof(float) * 3 * s->nn, S->pool) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&s->ev, hipEventDisableTiming) != hipSuccess) return false;
    float *Ms = s->par_dev, *A = s->par_dev + s->nc, *al = s->par_dev + 2 * s->nc;
    const size_t cb = sizeof(float) * s->nc;
    if (hipMemcpyAsync(Ms, s->Ms.data(), cb, hipMemcpyHostToDevice, s->stream) != hipSuccess) return false;
    if (hipMemcpyAsync(A, s->A.data(), cb, hipMemcpyHostToDevice, s->stream) != hipSuccess) return false;
    if (hipMemcpyAsync(al, s->alpha.data(), cb, hipMemcpyHostToDevice, s->stream) != hipSuccess) return false;
    if (hipMemcpyAsync(s->m_dev, s->m0.data(), sizeof(float) * 3 * s->nn, hipMemcpyHostToDevice, s->stream) !=
        hipSuccess)
        return false;
    nm_mesh_desc d{};
    for (int k = 0; k < 3; ++k) {
        d.n[k] = r.n[k];
        d.h[k] = r.h[k];
    }
    d.gamma = r.gamma;
    d.stream = s->stream;
    nm_material mat{};
    mat.Ms = Ms;
    mat.A = A;
    mat.alpha = al;
    for (int k = 0; k < 3; ++k) mat.h_uniform[k] = r.h_uniform[k];
    if (nm_mesh_create(&d, &mat, &s->mesh) != NM_OK) return false;
    if ((r.terms & NM_T_DEMAG) && nm_demag_tensor_init(s->mesh) != NM_OK) return false;
    nm_integrator in{};
    in.method = NM_DP45;
    in.terms = r.terms;
    in.rtol = r.rtol;
    in.atol = r.atol;
    in.dt_min = 1e-20;
    s->clk = nm_clock{0.0, r.dt0, 0, 0, 0, 0.0};
    if (step_begin(s->mesh, s->m_dev, &s->clk, &in, r.t_end, 1L << 40, &s->batch) != NM_OK) return false;
    s->batch = S->desc.attempts_per_launch;
    s->next = batch_for(std::ceil(r.t_end / r.dt0 * (1.0 + 1e-9)), s->batch);
    s->res.t_admit = now_s();
    return true;
}

void complete(nm_server *S, Solve *s) {
    nm_status st = step_finish(s->mesh, NM_DP45, &s->clk);
    s->m_out.resize(3 * s->nn);
    hipError_t e = hipMemcpyAsync(s->m_out.data(), s->m_dev, sizeof(float) * 3 * s->nn,
                                  hipMemcpyDeviceToHost, s->stream);
    // wait for this solve's work only (the stream is shared with other solves)
    if (e == hipSuccess) e = hipEventRecord(s->ev, s->stream);
    if (e == hipSuccess) e = hipEventSynchronize(s->ev);
    s->res.status = e != hipSuccess ? NM_EHIP : st;
    s->res.t = s->clk.t;
    s->res.accepted = s->clk.accepted;
    s->res.rejected = s->clk.rejected;
    s->res.rhs_evals = s->clk.rhs_evals;
    release(s, S->pool);
    s->res.t_done = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    S->used -= s->footprint;
    S->done[s->ticket] = s;
    S->known[s->ticket] = 2;
    S->cv_done.notify_all();
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
                if (S->active.empty() && S->pending.empty()) {
                    S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
                    if (S->stop) return;
                }
                if (S->pending.empty() || (int)S->active.size() >= S->desc.max_active) break;
                Solve *f = S->pending.front();
                if (S->used + f->footprint > S->budget) {
                    if (!S->active.empty()) break;   // wait for memory to free up
                    S->pending.pop_front();          // can never fit
                    lk.unlock();
                    fail(S, f, NM_EBUDGET);
                    continue;
                }
                S->pending.pop_front();
                S->used += f->footprint;
                S->known[f->ticket] = 1;
                s = f;
            }
            if (!admit(S, s)) {
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->used -= s->footprint;
                }
                fail(S, s, NM_EHIP);
                continue;
            }
            S->active.push_back(s);
        }
        // issue a replay for every idle solve, retire finished ones
        bool progressed = false;
        for (Solve *s : S->active) {
            if (s->inflight) continue;
            hipError_t e = step_batch(s->mesh, s->m_dev, NM_DP45, s->req.terms, s->batch, s->next);
            if (e == hipSuccess) e = ctrl_readback(s->mesh);
            if (e == hipSuccess) e = hipEventRecord(s->ev, s->stream);
            if (e != hipSuccess) {
                s->res.status = NM_EHIP;
                s->inflight = false;
                continue;
            }
            s->inflight = true;
            progressed = true;
        }
        std::vector<Solve *> still;
        for (Solve *s : S->active) {
            if (s->res.status == NM_EHIP) {
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    S->used -= s->footprint;
                }
                fail(S, s, NM_EHIP);
                progressed = true;
                continue;
            }
            if (s->inflight && hipEventQuery(s->ev) == hipSuccess) {
                s->inflight = false;
                progressed = true;
                if (s->mesh->ctrl_host->done) {
                    complete(S, s);
                    continue;
                }
                s->next = next_batch(s->mesh, s->batch);
            }
            still.push_back(s);
        }
        S->active.swap(still);
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
    for (int i = 0; i < desc->n_streams; ++i) {
        hipStream_t st = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
            delete S;
            set_error("nm_server_create: stream creation failed");
            return NM_EHIP;
        }
        S->streams.push_back(st);
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
    for (Solve *s : S->active) {
        (void)hipStreamSynchronize(s->stream);
        release(s, S->pool);
        delete s;
    }
    for (Solve *s : S->pending) delete s;
    for (auto &kv : S->done) delete kv.second;
    for (hipStream_t x : S->streams) (void)hipStreamDestroy(x);
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
    const size_t fp = solve_footprint(*r);
    NM_REQUIRE(fp > 0, NM_EINVAL, "nm_serve_submit: unsupported mesh size");
    Solve *s = new Solve();
    s->req = *r;
    s->footprint = fp;
    const size_t nc = (size_t)r->n[0] * r->n[1] * r->n[2];
    const size_t nn = (size_t)(r->n[0] + 1) * (r->n[1] + 1) * (r->n[2] + 1);
    s->Ms.assign(r->Ms, r->Ms + nc);
    s->A.assign(r->A, r->A + nc);
    s->alpha.assign(r->alpha, r->alpha + nc);
    s->m0.assign(r->m0, r->m0 + 3 * nn);
    s->req.Ms = s->req.A = s->req.alpha = s->req.m0 = nullptr;
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
