// Demagnetisation tensor set-up in float64 (Sec. 3.2), gfx950.
//
// N(d) is the cell-averaged field of a homogeneously magnetised cuboid cell
// at integer cell offset d (H_c = -sum N(c - c') M_c').  Near the source the
// closed form of Newell, Williams and Dunlop (J. Geophys. Res. 98, 9551,
// 1993) is used: N = D f / (4 pi V), D the 27-point second difference over
// the cell edges, f / g the Newell potentials.  It cancels catastrophically
// with distance (about (r/h)^6 digits), so further out N is evaluated from
// its integral definition,
//     N(X) = int_{[-h,h]^3} prod_k (1 - |u_k|/h_k) N_dip(X + u) du,
//     N_dip(r) = (delta r^2 - 3 r r^T) / (4 pi r^5),
// by tensor Gauss-Legendre quadrature on each half axis (the kink of the
// tent is at u = 0); the number of points falls with distance.
//
// The k-space tensor is real: the diagonal components are even along every
// axis and each off-diagonal one is odd along exactly two axes, so the DFT of
// the zero-padded tensor reduces to separable cosine / sine sums over the
// non-negative octant of offsets.  Those sums run in float64 here; the result
// is stored in float32 on the half spectrum 0 <= ky <= P2/2, 0 <= kz <= P3/2
// (the rest follows by parity) and carries the 1/(P1 P2 P3) of the inverse.
#include <cmath>
#include <mutex>
#include <string>

#include "nm_internal.h"

namespace nm {

namespace {

constexpr double kPi = 3.14159265358979323846;

// distance bands (in units of the longest cell edge) and Gauss-Legendre
// points per half axis; Newell below the first edge
constexpr double kNearRadius = 3.5;
constexpr int kBands = 5;
constexpr double kBandEdge[kBands] = {6.0, 12.0, 30.0, 80.0, 1e300};
constexpr int kBandPts[kBands] = {8, 6, 5, 4, 3};
constexpr int kMaxPts = 8;

struct TentRules {
    // per band and axis: 2 * npts nodes and weights of the tent-weighted rule
    double u[kBands][3][2 * kMaxPts];
    double w[kBands][3][2 * kMaxPts];
};

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double t = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) {
                // recompute the derivative at the converged node for the weight
                p0 = 1.0;
                p1 = t;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                const double d = n * (t * p1 - p0) / (t * t - 1.0);
                x[i] = t;
                w[i] = 2.0 / ((1.0 - t * t) * d * d);
                break;
            }
        }
    }
}

__device__ __forceinline__ double q_ratio(double num, double den) { return den != 0.0 ? num / den : 0.0; }

// Newell potential for the diagonal components (even in each argument)
__device__ double newell_f(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = (2.0 * x2 - y2 - z2) * R / 6.0;
    const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
    if (rxz > 0.0) r += 0.5 * y * (z2 - x2) * asinh(y / rxz);
    if (rxy > 0.0) r += 0.5 * z * (y2 - x2) * asinh(z / rxy);
    if (x != 0.0) r -= x * y * z * atan(q_ratio(y * z, x * R));
    return r;
}

// Newell potential for the xy component (odd in x and y)
__device__ double newell_g(double x, double y, double z) {
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double R = sqrt(x2 + y2 + z2);
    double r = -x * y * R / 3.0;
    const double rxy = sqrt(x2 + y2), ryz = sqrt(y2 + z2), rxz = sqrt(x2 + z2);
    if (rxy > 0.0) r += x * y * z * asinh(z / rxy);
    if (ryz > 0.0) r += y * (3.0 * z2 - y2) * asinh(x / ryz) / 6.0;
    if (rxz > 0.0) r += x * (3.0 * z2 - x2) * asinh(y / rxz) / 6.0;
    if (z != 0.0) r -= z * z2 * atan(q_ratio(x * y, z * R)) / 6.0;
    if (y != 0.0) r -= 0.5 * z * y2 * atan(q_ratio(x * z, y * R));
    if (x != 0.0) r -= 0.5 * z * x2 * atan(q_ratio(y * z, x * R));
    return r;
}

__device__ void tensor_near(double X, double Y, double Z, double h0, double h1, double h2,
                            double out[6]) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int e3 = -1; e3 <= 1; ++e3) {
        const double w3 = e3 == 0 ? 2.0 : -1.0, z = Z + e3 * h2;
        for (int e2 = -1; e2 <= 1; ++e2) {
            const double w2 = e2 == 0 ? 2.0 : -1.0, y = Y + e2 * h1;
            for (int e1 = -1; e1 <= 1; ++e1) {
                const double w = (e1 == 0 ? 2.0 : -1.0) * w2 * w3, x = X + e1 * h0;
                acc[0] += w * newell_f(x, y, z);
                acc[1] += w * newell_f(y, x, z);
                acc[2] += w * newell_f(z, y, x);
                acc[3] += w * newell_g(x, y, z);
                acc[4] += w * newell_g(x, z, y);
                acc[5] += w * newell_g(y, z, x);
            }
        }
    }
    const double s = 1.0 / (4.0 * kPi * h0 * h1 * h2);
    for (int c = 0; c < 6; ++c) out[c] = acc[c] * s;
}

__device__ void tensor_far(double X, double Y, double Z, const TentRules *__restrict__ R, int band,
                           double out[6]) {
    const int n2 = 2 * kBandPts[band];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int a = 0; a < n2; ++a) {
        const double x = X + R->u[band][0][a], wa = R->w[band][0][a];
        for (int b = 0; b < n2; ++b) {
            const double y = Y + R->u[band][1][b], wab = wa * R->w[band][1][b];
            for (int c = 0; c < n2; ++c) {
                const double z = Z + R->u[band][2][c], w = wab * R->w[band][2][c];
                const double r2 = x * x + y * y + z * z;
                const double k = w / (r2 * r2 * sqrt(r2));
                acc[0] += k * (r2 - 3.0 * x * x);
                acc[1] += k * (r2 - 3.0 * y * y);
                acc[2] += k * (r2 - 3.0 * z * z);
                acc[3] -= k * 3.0 * x * y;
                acc[4] -= k * 3.0 * x * z;
                acc[5] -= k * 3.0 * y * z;
            }
        }
    }
    for (int c = 0; c < 6; ++c) out[c] = acc[c] / (4.0 * kPi);
}

__global__ void k_newell_octant(int n1, int n2, int n3, double h0, double h1, double h2,
                                const TentRules *__restrict__ rules, double *__restrict__ out) {
    const long long total = (long long)n1 * n2 * n3;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int d1 = (int)(i % n1);
    const int d2 = (int)((i / n1) % n2);
    const int d3 = (int)(i / ((long long)n1 * n2));
    const double X = d1 * h0, Y = d2 * h1, Z = d3 * h2;
    const double rho = sqrt(X * X + Y * Y + Z * Z);  // edges scaled so the longest is 1
    double v[6];
    if (rho < kNearRadius) {
        tensor_near(X, Y, Z, h0, h1, h2, v);
    } else {
        int band = 0;
        while (band < kBands - 1 && rho >= kBandEdge[band]) ++band;
        tensor_far(X, Y, Z, rules, band, v);
    }
    for (int c = 0; c < 6; ++c) out[c * total + i] = v[c];
}

// parity of component c along axis a (1 = odd)
__host__ __device__ constexpr int odd_along(int c, int a) {
    return (c == 3 && a != 2) || (c == 4 && a != 1) || (c == 5 && a != 0);
}

// one axis of the separable transform:
// out[c][..][k][..] = sum_{d < nd} tau_c(k, d) in[c][..][d][..]
// with tau = (d ? 2 : 1) cos(2 pi k d / P) (even) or 2 sin(2 pi k d / P) (odd)
template <typename TOut>
__global__ void k_axis_transform(const double *__restrict__ in, TOut *__restrict__ out, int axis,
                                 int inner, int nd, int nk, int outer, int P,
                                 const double2 *__restrict__ cs, double final_scale) {
    const long long per = (long long)outer * nk * inner;
    const long long total = 6 * per;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int c = (int)(i / per);
    long long r = i - c * per;
    const int o = (int)(r / ((long long)nk * inner));
    r -= (long long)o * nk * inner;
    const int k = (int)(r / inner);
    const int q = (int)(r - (long long)k * inner);
    const bool odd = odd_along(c, axis);
    const double *src = in + ((long long)c * outer + o) * nd * inner + q;
    double acc = 0.0;
    for (int d = 0; d < nd; ++d) {
        const int ph = (int)(((long long)k * d) % P);
        const double2 e = cs[ph];
        const double wt = odd ? 2.0 * e.y : (d == 0 ? 1.0 : 2.0) * e.x;
        acc += wt * src[(long long)d * inner];
    }
    // two odd axes contribute (-i)^2 = -1 to every off-diagonal component
    const double sgn = (final_scale != 0.0 && c >= 3) ? -1.0 : 1.0;
    const double sc = final_scale != 0.0 ? final_scale : 1.0;
    out[i] = (TOut)(sgn * sc * acc);
}

}  // namespace

static void scaled_edges(const double h[3], double s[3]) {
    const double hm = std::fmax(h[0], std::fmax(h[1], h[2]));
    for (int k = 0; k < 3; ++k) s[k] = h[k] / hm;
}

// the tent-weighted rules of every band, built on the host in float64 and
// copied into the device buffer dev (synchronous on stream)
static hipError_t upload_rules(const double hs[3], TentRules *dev, hipStream_t stream) {
    TentRules host{};
    for (int b = 0; b < kBands; ++b) {
        const int n = kBandPts[b];
        double x[kMaxPts], w[kMaxPts];
        gauss_legendre(n, x, w);
        for (int a = 0; a < 3; ++a) {
            for (int i = 0; i < n; ++i) {
                const double u = 0.5 * (x[i] + 1.0) * hs[a];       // node on [0, h]
                const double wt = 0.5 * w[i] * hs[a] * (1.0 - u / hs[a]);
                host.u[b][a][i] = -u;
                host.w[b][a][i] = wt;
                host.u[b][a][n + i] = u;
                host.w[b][a][n + i] = wt;
            }
        }
    }
    hipError_t e = hipMemcpyAsync(dev, &host, sizeof(TentRules), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e;
}

// the octant into out with the rules in the device buffer rules
static hipError_t newell_octant_with(int n1, int n2, int n3, const double h[3], TentRules *rules, double *out,
                                     hipStream_t stream) {
    double hs[3];
    scaled_edges(h, hs);
    hipError_t e = upload_rules(hs, rules, stream);
    if (e != hipSuccess) return e;
    const long long total = (long long)n1 * n2 * n3;
    hipLaunchKernelGGL(k_newell_octant, dim3((unsigned)((total + 127) / 128)), dim3(128), 0, stream,
                       n1, n2, n3, hs[0], hs[1], hs[2], rules, out);
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(stream);
    return e != hipSuccess ? e : e2;
}

hipError_t launch_newell_octant(int n1, int n2, int n3, const double h[3], double *out,
                                hipStream_t stream) {
    TentRules *rules = nullptr;
    hipError_t e = dev_alloc((void **)&rules, sizeof(TentRules), thread_pool());
    if (e != hipSuccess) return e;
    e = newell_octant_with(n1, n2, n3, h, rules, out, stream);
    dev_free(rules, thread_pool());
    return e;
}

// cos and sin of 2 pi r / P, r < P (P <= kMaxFFT), into the device buffer dev
static hipError_t upload_phases(int P, double2 *dev, hipStream_t stream) {
    double2 cs[kMaxFFT];
    for (int r = 0; r < P; ++r) {
        const double a = 2.0 * kPi * r / P;
        cs[r] = make_double2(std::cos(a), std::sin(a));
    }
    hipError_t e = hipMemcpyAsync(dev, cs, sizeof(double2) * P, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e;
}

// Layout of the float64 temporaries of the k-space transform inside one
// scratch buffer: the octant [6][n3][n2][n1], the x transform
// [6][n3][n2][KP], the y transform [6][n3][P2h][KP], the phase tables of the
// three axes and the tent rules, each at a 256-byte boundary.
namespace {
struct KspaceScratch {
    size_t octd, A, B, c1, c2, c3, rules, total;
};
KspaceScratch kspace_layout(int N1, int N2, int N3, int P1, int P2, int P3) {
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t KP = (size_t)(P1 / 2 + 1 + 15) / 16 * 16, P2h = (size_t)P2 / 2 + 1;
    KspaceScratch L{};
    size_t off = 0;
    L.octd = off; off += up(sizeof(double) * 6 * (size_t)N1 * N2 * N3);
    L.A = off;    off += up(sizeof(double) * 6 * (size_t)N3 * N2 * KP);
    L.B = off;    off += up(sizeof(double) * 6 * (size_t)N3 * P2h * KP);
    L.c1 = off;   off += up(sizeof(double2) * (size_t)P1);
    L.c2 = off;   off += up(sizeof(double2) * (size_t)P2);
    L.c3 = off;   off += up(sizeof(double2) * (size_t)P3);
    L.rules = off; off += up(sizeof(TentRules));
    L.total = off;
    return L;
}
KspaceScratch kspace_layout(const nm_mesh *m) { return kspace_layout(m->N1, m->N2, m->N3, m->P1, m->P2, m->P3); }
}  // namespace

size_t kspace_scratch_bytes(const nm_mesh *m) { return kspace_layout(m).total; }
size_t kspace_scratch_bytes(int N1, int N2, int N3, int P1, int P2, int P3) {
    return kspace_layout(N1, N2, N3, P1, P2, P3).total;
}

// octant (float64) -> reduced k-space tensor (float32) for the mesh, with
// every temporary in the device buffer `work` (kspace_scratch_bytes(m) bytes,
// 256-byte aligned); allocates nothing
hipError_t build_kspace_tensor_with(nm_mesh *m, void *work) {
    const KspaceScratch L = kspace_layout(m);
    char *w = static_cast<char *>(work);
    double *octd = reinterpret_cast<double *>(w + L.octd);
    double *A = reinterpret_cast<double *>(w + L.A);
    double *B = reinterpret_cast<double *>(w + L.B);
    double2 *c1 = reinterpret_cast<double2 *>(w + L.c1);
    double2 *c2 = reinterpret_cast<double2 *>(w + L.c2);
    double2 *c3 = reinterpret_cast<double2 *>(w + L.c3);
    TentRules *rules = reinterpret_cast<TentRules *>(w + L.rules);
    const int n1 = m->N1, n2 = m->N2, n3 = m->N3;
    // x frequencies stored at the padded pitch KP (entries past K1 unused)
    const long long sa = 6LL * n3 * n2 * m->KP;
    const long long sb = 6LL * n3 * m->P2h * m->KP;
    hipError_t e = upload_phases(m->P1, c1, m->stream);
    if (e == hipSuccess) e = upload_phases(m->P2, c2, m->stream);
    if (e == hipSuccess) e = upload_phases(m->P3, c3, m->stream);
    if (e == hipSuccess) e = newell_octant_with(n1, n2, n3, m->h, rules, octd, m->stream);
    if (e != hipSuccess) return e;
    const int th = 128;
    // x: [6][n3][n2][n1] -> [6][n3][n2][KP]
    long long tot = sa;
    hipLaunchKernelGGL((k_axis_transform<double>), dim3((unsigned)((tot + th - 1) / th)), dim3(th),
                       0, m->stream, octd, A, 0, 1, n1, m->KP, n3 * n2, m->P1, c1, 0.0);
    // y: [6][n3][n2][KP] -> [6][n3][P2h][KP]
    tot = sb;
    hipLaunchKernelGGL((k_axis_transform<double>), dim3((unsigned)((tot + th - 1) / th)), dim3(th),
                       0, m->stream, A, B, 1, m->KP, n2, m->P2h, n3, m->P2, c2, 0.0);
    // z: [6][n3][P2h][KP] -> [6][P3h][P2h][KP], sign and 1/(P1 P2 P3)
    tot = 6LL * m->P3h * m->P2h * m->KP;
    const double scale = 1.0 / ((double)m->P1 * m->P2 * m->P3);
    hipLaunchKernelGGL((k_axis_transform<float>), dim3((unsigned)((tot + th - 1) / th)), dim3(th),
                       0, m->stream, B, m->tensor, 2, m->P2h * m->KP, n3, m->P3h, 1, m->P3, c3,
                       scale);
    e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(m->stream);
    return e != hipSuccess ? e : e2;
}

// the same with the temporaries taken from the mesh's allocator hooks if it
// has them, else from the calling thread's pool if it has one (no
// device-wide wait when they are given back), else hipMalloc
hipError_t build_kspace_tensor(nm_mesh *m) {
    DevPool *pool = m->owns_pool ? m->pool : thread_pool();
    void *work = nullptr;
    hipError_t e = dev_alloc(&work, kspace_scratch_bytes(m), pool);
    if (e != hipSuccess) return e;
    e = build_kspace_tensor_with(m, work);
    dev_free(work, pool);
    return e;
}

// --------------------------------------------- set-up without allocation
// Callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid it) initialise the tensor with
// nm_demag_tensor_init_noalloc, whose float64 temporaries live in this
// file-scope array: kNoAllocScratch bytes on every device the library runs
// on, held until the process ends.  In host code the array's name only
// stands in for it; the device address of each device's copy comes from
// hipGetSymbolAddress (once per device, with that device current) and is the
// only form passed to kernels and copies.
constexpr size_t kNoAllocScratch = size_t(96) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];   // one call at a time per device
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

}  // namespace nm

extern "C" nm_status nm_demag_tensor_init_noalloc(nm_mesh *m) {
    using namespace nm;
    if (!m) {
        set_error("nm_demag_tensor_init_noalloc: NULL mesh");
        return NM_EINVAL;
    }
    if (m->tensor_ready) return NM_OK;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != m->device || dev < 0 || dev >= kMaxDevices) {
        set_error("nm_demag_tensor_init_noalloc: the mesh's device must be the current device");
        return NM_EINVAL;
    }
    const size_t need = kspace_scratch_bytes(m);
    if (need > kNoAllocScratch) {
        set_error("nm_demag_tensor_init_noalloc: the tensor set-up of this grid needs " + std::to_string(need) +
                  " bytes of scratch, more than the " + std::to_string(kNoAllocScratch) +
                  " this entry point has; use nm_demag_tensor_init");
        return NM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            set_error(std::string("nm_demag_tensor_init_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
            return NM_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    // every temporary is written in full before it is read: nothing to clear
    const hipError_t e = build_kspace_tensor_with(m, g_scratch_ptr[dev]);
    if (e != hipSuccess) {
        set_error(std::string("nm_demag_tensor_init_noalloc: ") + hipGetErrorString(e));
        return NM_EHIP;
    }
    // the tile widths stay as they are (the tuner would create timing events)
    m->tensor_ready = true;
    return NM_OK;
}
