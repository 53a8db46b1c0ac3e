// C ABI of the library: mesh lifetime, argument checks and the drivers of the
// field, energy and time-stepping kernels.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nm_internal.h"

namespace nm {

static thread_local std::string g_error;

void set_error(const std::string &msg) { g_error = msg; }

static std::mutex g_tw_mutex;
static std::map<int, float2 *> g_tw;

// exp(-2 pi i t / kTwN), built in float64 on the host, one table per device
const float2 *twiddles(int device) {
    std::lock_guard<std::mutex> lock(g_tw_mutex);
    auto it = g_tw.find(device);
    if (it != g_tw.end()) return it->second;
    std::vector<float2> host(kTwN);
    const double pi = 3.14159265358979323846;
    for (int t = 0; t < kTwN; ++t) {
        const double a = -2.0 * pi * t / kTwN;
        host[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    float2 *dev = nullptr;
    if (hipMalloc(&dev, sizeof(float2) * kTwN) != hipSuccess) return nullptr;
    if (hipMemcpy(dev, host.data(), sizeof(float2) * kTwN, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(dev);
        return nullptr;
    }
    g_tw[device] = dev;
    return dev;
}

// ------------------------------------------------------------- set-up kernels
__global__ void k_cell_setup(const float *__restrict__ Ms, const float *__restrict__ A,
                             float *__restrict__ wc, float *__restrict__ A2, long long nc, float w) {
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    wc[c] = w * Ms[c];
    A2[c] = 2.f * A[c];
}

// M_n = mu0 sum_{c containing n} Ms_c V/8 (Eq. mass_lumping); Ms-weighted damping.
// Under the film basis the single node layer sits at z = 0: its 4 cells give
// half the film mass, consistent with the node kernel's gradient there (the
// field -g/M is the film's).
// cubic anisotropy per cell, packed for the node kernel: {Kc, c1}, {c2, 0}
__global__ void k_cubic_pack(const float *__restrict__ Kc, const float *__restrict__ ax,
                             float4 *__restrict__ out, long long nc) {
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    out[2 * c] = make_float4(Kc[c], ax[c], ax[nc + c], ax[2 * nc + c]);
    out[2 * c + 1] = make_float4(ax[3 * nc + c], ax[4 * nc + c], ax[5 * nc + c], 0.f);
}

__global__ void k_node_setup(const float *__restrict__ Ms, const float *__restrict__ alpha,
                             const float *__restrict__ wc, float *__restrict__ inv_mass,
                             float *__restrict__ alpha_n, float *__restrict__ gp_n, int N1, int N2,
                             int N3, int NZ, double gamma) {
    const int NX = N1 + 1, NY = N2 + 1;
    const long long nn = (long long)NX * NY * NZ;
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    const int x = (int)(n % NX), y = (int)((n / NX) % NY), z = (int)(n / ((long long)NX * NY));
    double M = 0.0, sa = 0.0, sm = 0.0;
    for (int i3 = 0; i3 < 2; ++i3)
        for (int i2 = 0; i2 < 2; ++i2)
            for (int i1 = 0; i1 < 2; ++i1) {
                const int cx = x - i1, cy = y - i2, cz = z - i3;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= N1 || cy >= N2 || cz >= N3) continue;
                const long long c = ((long long)cz * N2 + cy) * N1 + cx;
                M += wc[c];
                sm += Ms[c];
                sa += (double)Ms[c] * alpha[c];
            }
    const double a = sm > 0.0 ? sa / sm : 0.0;
    inv_mass[n] = M > 0.0 ? (float)(1.0 / M) : 0.f;
    alpha_n[n] = (float)a;
    gp_n[n] = (float)(gamma / (1.0 + a * a));
}

}  // namespace nm

using namespace nm;

#define NM_REQUIRE(cond, code, msg)  \
    do {                             \
        if (!(cond)) {               \
            set_error(msg);          \
            return code;             \
        }                            \
    } while (0)

#define NM_HIP(call, what)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            set_error(std::string(what) + ": " + hipGetErrorString(e_));            \
            return e_ == hipErrorOutOfMemory ? NM_ENOMEM : NM_EHIP;                 \
        }                                                                           \
    } while (0)

static int pad_len(int n) {
    if (n <= 1) return 1;
    int p = 1;
    while (p < 2 * n - 1) p <<= 1;
    return p;
}

struct Sizes {
    int P1, P2, P3, K1, KP, P2h, P3h;
    long long nn, nc, spec, tensor, partials, eblocks;
};

static bool sizes_of(const nm_mesh_desc *d, Sizes *s) {
    const int n1 = d->n[0], n2 = d->n[1], n3 = d->n[2];
    if (n1 < 2 || n2 < 2 || n3 < 1) return false;
    if (d->basis != NM_BASIS_3D && d->basis != NM_BASIS_FILM) return false;
    if (d->basis == NM_BASIS_FILM && n3 != 1) return false;
    s->P1 = pad_len(n1);
    s->P2 = pad_len(n2);
    s->P3 = pad_len(n3);
    if (s->P1 > kMaxFFT || s->P2 > kMaxFFT || s->P3 > kMaxFFT) return false;
    s->K1 = s->P1 / 2 + 1;
    s->KP = (s->K1 + 15) / 16 * 16;
    s->P2h = s->P2 / 2 + 1;
    s->P3h = s->P3 / 2 + 1;
    s->nn = (long long)(n1 + 1) * (n2 + 1) * (d->basis == NM_BASIS_FILM ? 1 : n3 + 1);
    s->nc = (long long)n1 * n2 * n3;
    s->spec = 3LL * n3 * s->P2 * s->KP;
    s->tensor = 6LL * s->P3h * s->P2h * s->KP;
    s->partials = (s->nn + 255) / 256;   // one DP45 error partial per node block
    s->eblocks = (s->nc + 255) / 256;
    return true;
}

static size_t footprint(const Sizes &s) {
    size_t b = 0;
    b += sizeof(float) * s.nc * (1 + 1 + 1 + 1 + 3 + 3 + 1 + 1);  // Ms, A2, wc, Ku, easy, h_cell, drive, D
    b += sizeof(float) * s.nc * (4 + 4 + 8);                  // cellP, wstat, cubic
    b += sizeof(float) * s.nn * 3;                              // inv_mass, alpha_n, gp_n
    b += sizeof(float2) * s.spec + sizeof(float) * s.tensor;
    b += sizeof(float) * 4 * s.nc;                              // demag cell field / source
    b += sizeof(float) * 3 * s.nn * 11;                         // y[2], acc, k[7], RK4 compensation
    b += sizeof(Ctrl) + sizeof(ErrPartial) * s.partials + sizeof(double) * (5 * s.eblocks + 5);
    return b;
}

// Destroy the recorded graphs.  wait: a replay may still be queued on the
// mesh stream (RK4 calls return without waiting), so let it finish first;
// callers that know the stream is idle pass false.
static void drop_graph(nm_mesh *m, bool wait = true) {
    bool any = m->gexec != nullptr;
    for (hipGraphExec_t g : m->gtail) any = any || g != nullptr;
    if (any && wait) (void)hipStreamSynchronize(m->stream);
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    for (hipGraphExec_t &g : m->gtail) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
    m->gexec = nullptr;
    m->g_method = 0;
    m->g_terms = 0;
    m->g_mag = nullptr;
    m->g_batch = 0;
}

static void drop_adj_graph(nm_mesh *m, bool wait = true) {
    if ((m->adj_gexec || m->cadj_gexec) && wait) (void)hipStreamSynchronize(m->stream);
    if (m->adj_gexec) (void)hipGraphExecDestroy(m->adj_gexec);
    if (m->cadj_gexec) (void)hipGraphExecDestroy(m->cadj_gexec);
    m->adj_gexec = nullptr;
    m->cadj_gexec = nullptr;
}

// the mesh's stream work must be complete (nm_mesh_destroy waits for it,
// mesh_release callers guarantee it)
static void free_mesh(nm_mesh *m) {
    if (!m) return;
    prof_free(m);
    drop_graph(m, false);
    drop_adj_graph(m, false);
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    void *ptrs[] = {m->Ms, m->A2, m->Ku, m->easy, m->h_cell, m->drive_mask, m->Dc, m->wc, m->inv_mass,
                    m->alpha_n, m->gp_n, m->spec, m->tensor, m->hd, m->y[0], m->y[1], m->acc,
                    m->ctrl, m->partials, m->ered, m->cellP, m->wstat, m->cubP, m->mlo};
    for (void *p : ptrs) dev_free(p, m->pool);
    for (int j = 0; j < 7; ++j) dev_free(m->k[j], m->pool);
    host_free(m->ctrl_host, m->pool);
    if (m->owns_pool) pool_destroy(m->pool);
    delete m;
}

// release a mesh whose stream work is known to be complete (no stream wait)
void nm::mesh_release(nm_mesh *m) { free_mesh(m); }

template <typename T>
static hipError_t dalloc(nm_mesh *m, T **p, long long count) {
    return dev_alloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1), m->pool);
}

extern "C" size_t nm_mesh_footprint_bytes(const nm_mesh_desc *desc, int integrator) {
    (void)integrator;
    Sizes s;
    if (!desc || !sizes_of(desc, &s)) return 0;
    return footprint(s);
}

extern "C" nm_status nm_mesh_create(const nm_mesh_desc *d, const nm_material *mat, nm_mesh **out) {
    NM_REQUIRE(d && mat && out, NM_EINVAL, "nm_mesh_create: NULL argument");
    *out = nullptr;
    Sizes s;
    NM_REQUIRE(sizes_of(d, &s), NM_EINVAL,
               "nm_mesh_create: need n[0], n[1] >= 2, n[2] >= 1 (= 1 for the film basis), a known basis "
               "and padded lengths <= 1024");
    for (int k = 0; k < 3; ++k)
        NM_REQUIRE(std::isfinite(d->h[k]) && d->h[k] > 0.0, NM_EINVAL, "nm_mesh_create: h must be > 0");
    NM_REQUIRE(std::isfinite(d->gamma) && d->gamma > 0.0, NM_EINVAL, "nm_mesh_create: gamma must be > 0");
    NM_REQUIRE(mat->Ms && mat->A && mat->alpha, NM_EINVAL, "nm_mesh_create: Ms, A and alpha are required");
    NM_REQUIRE((d->alloc.alloc == nullptr) == (d->alloc.free == nullptr), NM_EINVAL,
               "nm_mesh_create: allocator hooks alloc and free must be given together");
    NM_REQUIRE((mat->Ku == nullptr) == (mat->easy == nullptr), NM_EINVAL,
               "nm_mesh_create: Ku and easy must be given together");
    NM_REQUIRE((mat->Kc == nullptr) == (mat->cubic == nullptr), NM_EINVAL,
               "nm_mesh_create: Kc and cubic must be given together");
    NM_REQUIRE(mat->dmi_type == NM_DMI_INTERFACIAL || mat->dmi_type == NM_DMI_BULK, NM_EINVAL,
               "nm_mesh_create: unknown dmi_type");
    NM_REQUIRE(std::isfinite(mat->drive_freq) && std::isfinite(mat->drive_phase), NM_EINVAL,
               "nm_mesh_create: non-finite drive parameters");

    nm_mesh *m = new nm_mesh();
    std::memset(m, 0, sizeof(nm_mesh));
    m->N1 = d->n[0];
    m->N2 = d->n[1];
    m->N3 = d->n[2];
    m->NX = m->N1 + 1;
    m->NY = m->N2 + 1;
    // the film basis keeps one node layer: every kernel reads the node layer
    // above a cell (z + 1) at z, which makes m constant along z
    m->NZ = d->basis == NM_BASIS_FILM ? 1 : m->N3 + 1;
    m->P1 = s.P1;
    m->P2 = s.P2;
    m->P3 = s.P3;
    m->K1 = s.K1;
    m->KP = s.KP;
    m->P2h = s.P2h;
    m->P3h = s.P3h;
    for (int k = 0; k < 3; ++k) m->h[k] = d->h[k];
    m->V = d->h[0] * d->h[1] * d->h[2];
    m->gamma = d->gamma;
    m->n_nodes = s.nn;
    m->n_cells = s.nc;
    m->stream = (hipStream_t)d->stream;
    m->n_partials = (int)s.partials;
    m->n_eblocks = (int)s.eblocks;
    m->has_anis = mat->Ku != nullptr;
    m->has_hcell = mat->h_cell != nullptr;
    m->has_drive = mat->drive_mask != nullptr;
    m->has_dmi = mat->D != nullptr;
    m->dmi_bulk = mat->dmi_type == NM_DMI_BULK;
    m->has_cubic = mat->Kc != nullptr;
    for (int k = 0; k < 3; ++k) {
        m->h_uniform[k] = mat->h_uniform[k];
        m->drive_amp[k] = mat->drive_amp[k];
    }
    m->drive_freq = mat->drive_freq;
    m->drive_phase = mat->drive_phase;

    // neighbour weights of the node kernel from the element matrices (terms.hip)
    {
        ElementTables T;
        std::string why;
        if (!generate_element_tables(d->h, &T, &why)) {
            delete m;
            set_error("nm_mesh_create: term generator: " + why);
            return NM_EINVAL;
        }
        for (int i = 0; i < 8; ++i) {
            m->Kp[i] = T.Kp[i];
            m->Mp[i] = T.Mp[i];
        }
        for (int i = 0; i < 4; ++i) {
            m->gx[i] = T.gx[i];
            m->gy[i] = T.gy[i];
            m->gz[i] = T.gz[i];
        }
        m->gq[0] = T.gq[0];
        m->gq[1] = T.gq[1];
        m->gw = T.gw;
    }

    m->owns_pool = d->alloc.alloc != nullptr;
    m->pool = m->owns_pool ? pool_create_user(d->alloc) : thread_pool();
    hipError_t e = hipGetDevice(&m->device);
    // the per-device twiddle table is built here, never inside a graph capture
    if (e == hipSuccess && !twiddles(m->device)) e = hipErrorOutOfMemory;
    const long long nc = s.nc, nn = s.nn;
    if (e == hipSuccess) e = dalloc(m, &m->Ms, nc);
    if (e == hipSuccess) e = dalloc(m, &m->A2, nc);
    if (e == hipSuccess) e = dalloc(m, &m->wc, nc);
    if (e == hipSuccess) e = dalloc(m, &m->h_cell, 3 * nc);
    if (e == hipSuccess) e = dalloc(m, &m->cellP, nc);
    if (e == hipSuccess) e = dalloc(m, &m->wstat, nc);
    if (e == hipSuccess && m->has_anis) e = dalloc(m, &m->Ku, nc);
    if (e == hipSuccess && m->has_anis) e = dalloc(m, &m->easy, 3 * nc);
    if (e == hipSuccess && m->has_drive) e = dalloc(m, &m->drive_mask, nc);
    if (e == hipSuccess && m->has_dmi) e = dalloc(m, &m->Dc, nc);
    if (e == hipSuccess && m->has_cubic) e = dalloc(m, &m->cubP, 2 * nc);
    if (e == hipSuccess) e = dalloc(m, &m->inv_mass, nn);
    if (e == hipSuccess) e = dalloc(m, &m->alpha_n, nn);
    if (e == hipSuccess) e = dalloc(m, &m->gp_n, nn);
    if (e == hipSuccess) e = dalloc(m, &m->spec, s.spec);
    if (e == hipSuccess) e = dalloc(m, &m->tensor, s.tensor);
    if (e == hipSuccess) e = dalloc(m, &m->hd, 4 * nc);
    if (e == hipSuccess) e = dalloc(m, &m->y[0], 3 * nn);
    if (e == hipSuccess) e = dalloc(m, &m->y[1], 3 * nn);
    if (e == hipSuccess) e = dalloc(m, &m->acc, 3 * nn);
    for (int j = 0; j < 7 && e == hipSuccess; ++j) e = dalloc(m, &m->k[j], 3 * nn);
    if (e == hipSuccess) e = dalloc(m, &m->mlo, 3 * nn);
    if (e == hipSuccess) e = dalloc(m, &m->ctrl, 1);
    if (e == hipSuccess) e = dalloc(m, &m->partials, s.partials);
    if (e == hipSuccess) e = dalloc(m, &m->ered, 5 * s.eblocks + 5);
    if (e == hipSuccess) e = host_alloc((void **)&m->ctrl_host, sizeof(Ctrl), m->pool);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        set_error(std::string("nm_mesh_create: allocation failed: ") + hipGetErrorString(e));
        free_mesh(m);
        return NM_ENOMEM;
    }
    hipStream_t st = m->stream;
    float *Atmp = m->A2;  // A is staged in A2 and doubled in place
    // the spectrum workspace starts zeroed: no pass writes the pitch's pad
    // columns (K1 <= kx < KP), and the column passes' pad lanes read them in
    // place, finite and in the same cache lines as their rows' last columns
    e = hipMemsetAsync(m->spec, 0, sizeof(float2) * (size_t)s.spec, st);
    if (e == hipSuccess) e = hipMemcpyAsync(m->Ms, mat->Ms, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(Atmp, mat->A, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && m->has_anis)
        e = hipMemcpyAsync(m->Ku, mat->Ku, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && m->has_anis)
        e = hipMemcpyAsync(m->easy, mat->easy, sizeof(float) * 3 * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && m->has_hcell)
        e = hipMemcpyAsync(m->h_cell, mat->h_cell, sizeof(float) * 3 * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && m->has_drive)
        e = hipMemcpyAsync(m->drive_mask, mat->drive_mask, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && m->has_dmi)
        e = hipMemcpyAsync(m->Dc, mat->D, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    // alpha is only needed here: stage it in acc (3 * nn >= nc floats)
    if (e == hipSuccess) e = hipMemcpyAsync(m->acc, mat->alpha, sizeof(float) * nc, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_cell_setup, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, m->Ms,
                           Atmp, m->wc, m->A2, nc, (float)(kMu0 * m->V / 8.0));
        hipLaunchKernelGGL(k_node_setup, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, m->Ms,
                           m->acc, m->wc, m->inv_mass, m->alpha_n, m->gp_n, m->N1, m->N2, m->N3,
                           m->NZ, m->gamma);
        if (m->has_cubic)
            hipLaunchKernelGGL(k_cubic_pack, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, mat->Kc,
                               mat->cubic, m->cubP, nc);
        e = hipGetLastError();
        if (e == hipSuccess) e = launch_cell_pack(m);
    }
    std::vector<float> im;
    if (e == hipSuccess) {
        im.resize(nn);
        e = hipMemcpyAsync(im.data(), m->inv_mass, sizeof(float) * nn, hipMemcpyDeviceToHost, st);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        set_error(std::string("nm_mesh_create: set-up failed: ") + hipGetErrorString(e));
        free_mesh(m);
        return NM_EHIP;
    }
    for (long long i = 0; i < nn; ++i) m->n_active += im[i] > 0.f;
    *out = m;
    return NM_OK;
}

extern "C" nm_status nm_mesh_destroy(nm_mesh *m) {
    if (!m) return NM_OK;
    (void)hipStreamSynchronize(m->stream);
    free_mesh(m);
    return NM_OK;
}

extern "C" nm_status nm_mesh_info(const nm_mesh *m, int64_t *n_nodes, int64_t *n_cells, int pad[3]) {
    NM_REQUIRE(m, NM_EINVAL, "nm_mesh_info: NULL mesh");
    if (n_nodes) *n_nodes = m->n_nodes;
    if (n_cells) *n_cells = m->n_cells;
    if (pad) {
        pad[0] = m->P1;
        pad[1] = m->P2;
        pad[2] = m->P3;
    }
    return NM_OK;
}

extern "C" nm_status nm_mesh_set_field(nm_mesh *m, const float *h_cell) {
    NM_REQUIRE(m, NM_EINVAL, "nm_mesh_set_field: NULL mesh");
    // recorded graphs stay valid: they read the repacked cell data from memory
    if (!h_cell) {
        m->has_hcell = false;
        NM_HIP(launch_cell_pack(m), "nm_mesh_set_field");
        return NM_OK;
    }
    NM_HIP(hipMemcpyAsync(m->h_cell, h_cell, sizeof(float) * 3 * m->n_cells, hipMemcpyDeviceToDevice,
                          m->stream),
           "nm_mesh_set_field");
    m->has_hcell = true;
    NM_HIP(launch_cell_pack(m), "nm_mesh_set_field");
    return NM_OK;
}

extern "C" nm_status nm_demag_tensor_init(nm_mesh *m) {
    NM_REQUIRE(m, NM_EINVAL, "nm_demag_tensor_init: NULL mesh");
    if (m->tensor_ready) return NM_OK;
    NM_HIP(build_kspace_tensor(m), "nm_demag_tensor_init");
    NM_HIP(tune_passes(m), "nm_demag_tensor_init");
    m->tensor_ready = true;
    return NM_OK;
}

extern "C" nm_status nm_mesh_tuning(nm_mesh *m, int set, int *y, int *z) {
    NM_REQUIRE(m && y && z, NM_EINVAL, "nm_mesh_tuning: NULL argument");
    if (set) {
        NM_REQUIRE(*y >= -1 && *y <= 2 && *z >= -1 && *z <= 2, NM_EINVAL,
                   "nm_mesh_tuning: widths are 0, 1, 2 (or -1 to keep)");
        if (*y >= 0) m->tune_y = *y;
        if (*z >= 0) m->tune_z = *z;
        drop_graph(m);
        drop_adj_graph(m);
    }
    *y = m->tune_y;
    *z = m->tune_z;
    return NM_OK;
}

extern "C" nm_status nm_newell_octant(const int n[3], const double h[3], double *out, void *stream) {
    NM_REQUIRE(n && h && out, NM_EINVAL, "nm_newell_octant: NULL argument");
    NM_REQUIRE(n[0] >= 1 && n[1] >= 1 && n[2] >= 1, NM_EINVAL, "nm_newell_octant: n must be >= 1");
    for (int k = 0; k < 3; ++k)
        NM_REQUIRE(std::isfinite(h[k]) && h[k] > 0.0, NM_EINVAL, "nm_newell_octant: h must be > 0");
    NM_HIP(launch_newell_octant(n[0], n[1], n[2], h, out, (hipStream_t)stream), "nm_newell_octant");
    return NM_OK;
}

static nm_status check_terms(nm_mesh *m, unsigned terms, const char *who) {
    if (terms & ~(unsigned)NM_T_ALL) {
        set_error(std::string(who) + ": unknown term bits");
        return NM_EINVAL;
    }
    if ((terms & NM_T_DEMAG) && !m->tensor_ready) {
        set_error(std::string(who) + ": NM_T_DEMAG needs nm_demag_tensor_init first");
        return NM_EINVAL;
    }
    return NM_OK;
}

static nm_status eval_nodes(nm_mesh *m, const float *mag, float *out, unsigned terms, double t,
                            int mode, const char *who) {
    NM_REQUIRE(m && mag && out, NM_EINVAL, std::string(who) + ": NULL argument");
    NM_REQUIRE(std::isfinite(t), NM_EINVAL, std::string(who) + ": non-finite time");
    nm_status st = check_terms(m, terms, who);
    if (st != NM_OK) return st;
    if (terms & NM_T_DEMAG)
        NM_HIP(demag_forward_conv_inverse(m, mag, (terms & NM_T_ZEEMAN) ? 2 : 1), who);
    StageSpec sp{};
    sp.mode = mode;
    sp.stage = 0;
    sp.in = mag;
    sp.out = out;
    sp.t0 = t;
    sp.use_ctrl = false;
    NM_HIP(launch_stencil(m, terms, sp), who);
    return NM_OK;
}

extern "C" nm_status nm_heff(nm_mesh *m, const float *mag, float *h, unsigned terms, double t) {
    return eval_nodes(m, mag, h, terms, t, kModeField, "nm_heff");
}

extern "C" nm_status nm_llg_rhs(nm_mesh *m, const float *mag, float *dmdt, unsigned terms, double t) {
    return eval_nodes(m, mag, dmdt, terms, t, kModeRhs, "nm_llg_rhs");
}

extern "C" nm_status nm_demag_cell_field(nm_mesh *m, const float *mag, float *hout) {
    NM_REQUIRE(m && mag && hout, NM_EINVAL, "nm_demag_cell_field: NULL argument");
    NM_REQUIRE(m->tensor_ready, NM_EINVAL, "nm_demag_cell_field: call nm_demag_tensor_init first");
    NM_HIP(demag_forward_conv_inverse(m, mag, 0), "nm_demag_cell_field");
    NM_HIP(hipMemcpyAsync(hout, m->hd, sizeof(float) * 3 * m->n_cells, hipMemcpyDeviceToDevice, m->stream),
           "nm_demag_cell_field");
    return NM_OK;
}

extern "C" nm_status nm_energy(nm_mesh *m, const float *mag, unsigned terms, double t, double e[6]) {
    NM_REQUIRE(m && mag && e, NM_EINVAL, "nm_energy: NULL argument");
    nm_status st = check_terms(m, terms, "nm_energy");
    if (st != NM_OK) return st;
    if (terms & NM_T_DEMAG) NM_HIP(demag_forward_conv_inverse(m, mag, 0), "nm_energy");
    NM_HIP(launch_energy(m, mag, terms, t, e), "nm_energy");
    return NM_OK;
}

// --------------------------------------------------------------- stepping
namespace {

hipError_t stage(nm_mesh *m, unsigned terms, int mode, int s, const float *in, float *y_next,
                 float *mstate, float *lo = nullptr) {
    if (terms & NM_T_DEMAG) {
        hipError_t e = demag_forward_conv_inverse_ctrl(m, in, m->ctrl, (terms & NM_T_ZEEMAN) ? 2 : 1);
        if (e != hipSuccess) return e;
    }
    StageSpec sp{};
    sp.mode = mode;
    sp.stage = s;
    sp.in = in;
    sp.y_next = y_next;
    sp.mstate = mstate;
    sp.use_ctrl = true;
    sp.lo = lo;
    return launch_stencil(m, terms, sp);
}

// DP45 stage s reads y_s from y[s % 2] (stage 1 reads the state) and writes
// y_{s+1} to y[(s + 1) % 2]
hipError_t dp45_stage(nm_mesh *m, unsigned terms, int s, const float *in, float *mstate) {
    return stage(m, terms, kModeDP45, s, in, s < 7 ? m->y[(s + 1) % 2] : nullptr, mstate);
}

// the state update (stage 4) carries its rounding error in m->mlo
hipError_t rk4_stage(nm_mesh *m, unsigned terms, int s, const float *in, float *y_next, float *mstate) {
    return stage(m, terms, kModeRK4, s, in, y_next, mstate, s == 4 ? m->mlo : nullptr);
}

}  // namespace

namespace nm {

// Controller initialisation from a kernel argument: the values travel with
// the launch, so a call may return while it is still queued (an asynchronous
// copy from host memory would race with the next call filling that memory).
__global__ void k_zero(float *__restrict__ p, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

__global__ void k_ctrl_set(Ctrl *C, Ctrl v) {
    const unsigned *src = reinterpret_cast<const unsigned *>(&v);
    unsigned *dst = reinterpret_cast<unsigned *>(C);
    for (unsigned i = threadIdx.x; i < sizeof(Ctrl) / 4; i += blockDim.x) dst[i] = src[i];
}

// Validate, initialise the device controller and, for DP45, launch the first
// stage.  *batch gets the number of steps / attempts one replay of the
// stepping graph covers.
nm_status step_begin(nm_mesh *m, float *mag, const nm_clock *clk, const nm_integrator *in,
                     double t_end, long max_steps, int *batch) {
    NM_REQUIRE(m && mag && clk && in, NM_EINVAL, "nm_llg_step: NULL argument");
    NM_REQUIRE(in->method == NM_RK4 || in->method == NM_DP45, NM_EINVAL, "nm_llg_step: unknown method");
    NM_REQUIRE(std::isfinite(clk->t) && std::isfinite(t_end) && t_end >= clk->t, NM_EINVAL,
               "nm_llg_step: need finite t <= t_end");
    NM_REQUIRE(std::isfinite(clk->dt) && clk->dt > 0.0, NM_EINVAL, "nm_llg_step: clk->dt must be > 0");
    NM_REQUIRE(max_steps > 0, NM_EINVAL, "nm_llg_step: max_steps must be > 0");
    if (in->method == NM_DP45)
        NM_REQUIRE(in->rtol > 0.0 && in->atol > 0.0, NM_EINVAL, "nm_llg_step: DP45 needs rtol, atol > 0");
    NM_REQUIRE(!in->log || in->log_capacity >= 0, NM_EINVAL, "nm_llg_step: bad log capacity");
    nm_status st = check_terms(m, in->terms, "nm_llg_step");
    if (st != NM_OK) return st;
    NM_REQUIRE(m->n_active > 0, NM_EINVAL, "nm_llg_step: the mesh has no magnetic node");
    Ctrl c0;
    Ctrl *C = &c0;
    std::memset(C, 0, sizeof(Ctrl));
    C->t = clk->t;
    C->dt_prop = clk->dt;
    C->dt = std::fmin(clk->dt, t_end - clk->t);
    C->t_end = t_end;
    C->rtol = in->rtol;
    C->atol = in->atol;
    C->dt_min = in->dt_min;
    C->dt_max = in->dt_max;
    C->stop_torque = in->stop_torque;
    C->norm_scale = 1.0 / (3.0 * (double)m->n_active);
    C->max_accepted = max_steps;
    C->log = in->log;
    C->log_cap = in->log ? in->log_capacity : 0;
    C->done = t_end == clk->t ? 1 : 0;
    static_assert(sizeof(Ctrl) % 4 == 0, "word copy");
    hipLaunchKernelGGL(k_ctrl_set, dim3(1), dim3(64), 0, m->stream, m->ctrl, c0);
    NM_HIP(hipGetLastError(), "nm_llg_step");
    // RK4 knows its step count: never capture more steps than the call needs
    int b = 16;
    if (in->method == NM_RK4) {
        // the compensation carries on only where the last RK4 call on this
        // mesh ended: the same state buffer at the clock it left behind
        if (!(m->lo_valid && m->lo_mag == mag && m->lo_t == clk->t)) {
            const long long n3 = 3 * m->n_nodes;
            hipLaunchKernelGGL(k_zero, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, m->stream, m->mlo, n3);
            NM_HIP(hipGetLastError(), "nm_llg_step");
        }
        const double span = (t_end - clk->t) / clk->dt;
        long need = (long)std::ceil(span * (1.0 - 1e-12));
        if (need > max_steps) need = max_steps;
        b = need < 8 ? (int)std::max(need, 1L) : 8;
    }
    *batch = b;
    // first DP45 stage (FSAL keeps k1 for every later attempt)
    if (in->method == NM_DP45) NM_HIP(dp45_stage(m, in->terms, 1, mag, mag), "nm_llg_step");
    return NM_OK;
}

// One batch of steps / attempts: launched directly while profiling, else
// replayed from a captured graph on the mesh stream.  The main graph holds
// `full` steps / attempts and is keyed on method, terms, state pointer and
// `full`; shorter power-of-two batches (the end of an integration) are
// captured beside it.  Every graph is uploaded right after instantiation,
// so its first replay costs what later ones cost.
static int tail_slot(int batch) {
    for (int k = 0; k < 6; ++k)
        if (batch == (1 << k)) return k;
    return -1;
}

int batch_for(double est, int batch) {
    if (est >= (double)batch) return batch;
    int b = 1;
    while (2 * b <= batch && (double)(2 * b) <= est) b *= 2;
    return b;
}

int next_batch(const nm_mesh *m, int batch) {
    const Ctrl *C = m->ctrl_host;
    double est = (double)(C->max_accepted - C->accepted);
    if (C->dt_prop > 0.0) est = std::fmin(est, std::ceil((C->t_end - C->t) / C->dt_prop * (1.0 + 1e-9)));
    return batch_for(est, batch);
}

hipError_t step_batch(nm_mesh *m, float *mag, int method, unsigned terms, int full, int batch) {
    auto enqueue_batch = [&](int count) -> hipError_t {
        hipError_t e = hipSuccess;
        for (int q = 0; q < count && e == hipSuccess; ++q) {
            if (method == NM_RK4) {
                if (e == hipSuccess) e = rk4_stage(m, terms, 1, mag, m->y[0], mag);
                if (e == hipSuccess) e = rk4_stage(m, terms, 2, m->y[0], m->y[1], mag);
                if (e == hipSuccess) e = rk4_stage(m, terms, 3, m->y[1], m->y[0], mag);
                if (e == hipSuccess) e = rk4_stage(m, terms, 4, m->y[0], nullptr, mag);
                if (e == hipSuccess) e = launch_rk4_advance(m);
            } else {
                for (int s = 2; s <= 7 && e == hipSuccess; ++s) e = dp45_stage(m, terms, s, m->y[s % 2], mag);
                if (e == hipSuccess) e = launch_dp45_control(m);
                if (e == hipSuccess) e = launch_dp45_finish(m, mag);
            }
        }
        return e;
    };
    if (m->prof) return enqueue_batch(batch);
    auto capture = [&](hipGraphExec_t *out, int count) -> hipError_t {
        hipStream_t user = m->stream;
        m->stream = m->cap_stream;
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed);
        hipError_t e2 = e == hipSuccess ? enqueue_batch(count) : e;
        if (e == hipSuccess) e = hipStreamEndCapture(m->cap_stream, &graph);
        m->stream = user;
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e == hipSuccess) e = hipGraphUpload(*out, m->stream);
        return e;
    };
    if (!(m->gexec && m->g_method == method && m->g_terms == terms && m->g_mag == mag && m->g_batch == full)) {
        drop_graph(m);
        hipError_t e = capture(&m->gexec, full);
        if (e != hipSuccess) return e;
        m->g_method = method;
        m->g_terms = terms;
        m->g_mag = mag;
        m->g_batch = full;
    }
    if (batch == full) return hipGraphLaunch(m->gexec, m->stream);
    const int ts = tail_slot(batch);
    if (ts < 0 || batch > full) return hipErrorInvalidValue;
    if (!m->gtail[ts]) {
        hipError_t e = capture(&m->gtail[ts], batch);
        if (e != hipSuccess) return e;
    }
    return hipGraphLaunch(m->gtail[ts], m->stream);
}

// asynchronous copy of the device controller into the pinned mirror
hipError_t ctrl_readback(nm_mesh *m) {
    return hipMemcpyAsync(m->ctrl_host, m->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, m->stream);
}

// fold the controller's counters into the caller's clock; map its status
nm_status step_finish(nm_mesh *m, int method, nm_clock *clk) {
    const Ctrl *C = m->ctrl_host;
    clk->t = C->t;
    if (method == NM_DP45) clk->dt = C->dt_prop;
    clk->accepted += C->accepted;
    clk->rejected += C->rejected;
    clk->rhs_evals += C->rhs_evals + (method == NM_DP45 ? 1 : 0);
    clk->max_torque = C->max_torque;
    if (C->status == NM_ENONFINITE) {
        set_error("nm_llg_step: non-finite error norm or state");
        return NM_ENONFINITE;
    }
    if (C->status == NM_ESTEPSIZE) {
        set_error("nm_llg_step: step size fell below dt_min");
        return NM_ESTEPSIZE;
    }
    return NM_OK;
}

}  // namespace nm

extern "C" nm_status nm_llg_step(nm_mesh *m, float *mag, nm_clock *clk, const nm_integrator *in,
                                 double t_end, long max_steps) {
    int batch = 1;
    nm_status st = step_begin(m, mag, clk, in, t_end, max_steps, &batch);
    if (st != NM_OK) return st;
    if (t_end == clk->t) return NM_OK;
    const unsigned terms = in->terms;
    if (in->method == NM_RK4) {
        const double span = (t_end - clk->t) / clk->dt;
        long nsteps = (long)std::ceil(span * (1.0 - 1e-12));
        if (nsteps < 1) nsteps = 1;
        if (nsteps > max_steps) nsteps = max_steps;
        for (long k = 0; k < nsteps;) {
            // the last replays take powers of two that add up to the rest
            const int b = batch_for((double)(nsteps - k), batch);
            NM_HIP(step_batch(m, mag, NM_RK4, terms, batch, b), "nm_llg_step");
            k += b;
        }
        // Fixed steps: the call returns without waiting for the GPU; the clock
        // advances on the host exactly as k_rk4_advance moves it on the device
        double t = clk->t, dt = std::fmin(clk->dt, t_end - clk->t);
        long acc = 0;
        for (;;) {
            const bool last = dt >= (t_end - t) * (1.0 - 1e-9);
            t = last ? t_end : t + dt;
            ++acc;
            if (last || acc >= max_steps) break;
            dt = std::fmin(clk->dt, t_end - t);
        }
        clk->t = t;
        clk->accepted += acc;
        clk->rhs_evals += 4 * acc;
        m->lo_valid = true;
        m->lo_mag = mag;
        m->lo_t = t;
        return NM_OK;
    } else {
        m->lo_valid = false;   // DP45 moves the state without the compensation
        long long seen = -1;
        int b = batch_for(std::fmin((double)max_steps, std::ceil((t_end - clk->t) / clk->dt * (1.0 + 1e-9))), batch);
        for (;;) {
            NM_HIP(step_batch(m, mag, NM_DP45, terms, batch, b), "nm_llg_step");
            NM_HIP(ctrl_readback(m), "nm_llg_step");
            NM_HIP(hipStreamSynchronize(m->stream), "nm_llg_step");
            if (m->ctrl_host->done) break;
            // every attempt either advances t or shrinks dt towards dt_min, so
            // the controller must make progress; anything else is a bug
            NM_REQUIRE(m->ctrl_host->attempts > seen, NM_EHIP, "nm_llg_step: controller made no progress");
            seen = m->ctrl_host->attempts;
            b = next_batch(m, batch);
        }
    }
    return step_finish(m, in->method, clk);
}

extern "C" const char *nm_last_error(void) { return g_error.c_str(); }
