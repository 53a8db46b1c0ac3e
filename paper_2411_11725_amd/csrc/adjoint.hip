// Discrete adjoint of fixed-step RK4 (Sec. 4: the gradient of a trajectory
// objective with respect to design variables, here the per-cell applied
// field map), with checkpointed recomputation of the forward states.
//
// For one RK4 step m -> m' with stages y_s, k_s = f(y_s, t_s) and the
// co-vector lam = dL/dm', the exact transpose runs the stages backwards
// with w_s the co-vector of k_s:
//   w4 = dt/6 lam, w3 = dt/3 lam + dt J4^T w4, w2 = dt/3 lam + dt/2 J3^T w3,
//   w1 = dt/6 lam + dt/2 J2^T w2,   dL/dm = lam + sum_s J_s^T w_s.
// J^T w of f(m, H(m)) splits into the node-local VJP of the LLG right-hand
// side and the transpose of the field; the linear part of the field is
// H_lin = -M^-1 K m with K symmetric, so (dH/dm)^T u = M H_lin(M^-1 u): the
// forward kernels evaluate it on the rescaled vector v = M^-1 u.  The field
// map enters as H_ext,n = sum_c (mu0 Ms_c V/8 / M_n) theta_c, so its gradient
// is the cell gather mu0 Ms_c V/8 sum_{n in c} v_n, accumulated over every
// stage and step first and gathered once.
#include <cmath>
#include <string>

#include "nm_internal.h"

namespace nm {

// u = df/dH^T w, vjp = df/dm^T w at (y, H); v = M^-1 u, vsum += v
__global__ void __launch_bounds__(256)
k_adj_vjp(const float *__restrict__ y, const float *__restrict__ H, const float *__restrict__ w,
          const float *__restrict__ inv_mass, const float *__restrict__ alpha_n,
          const float *__restrict__ gp_n, float *__restrict__ v, float *__restrict__ vjp,
          float *__restrict__ vsum, long long nn) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    float m[3], h[3], c[3];
    for (int k = 0; k < 3; ++k) {
        m[k] = y[k * nn + n];
        h[k] = H[k * nn + n];
        c[k] = w[k * nn + n];
    }
    const float a = gp_n[n], b = alpha_n[n] * gp_n[n], im = inv_mass[n];
    const float wm = c[0] * m[0] + c[1] * m[1] + c[2] * m[2];
    const float mh = m[0] * h[0] + m[1] * h[1] + m[2] * h[2];
    const float wh = c[0] * h[0] + c[1] * h[1] + c[2] * h[2];
    const float mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    const float hxw[3] = {h[1] * c[2] - h[2] * c[1], h[2] * c[0] - h[0] * c[2], h[0] * c[1] - h[1] * c[0]};
    const float mxw[3] = {m[1] * c[2] - m[2] * c[1], m[2] * c[0] - m[0] * c[2], m[0] * c[1] - m[1] * c[0]};
    for (int k = 0; k < 3; ++k) {
        const float dm = -a * hxw[k] - b * (h[k] * wm + mh * c[k] - 2.f * m[k] * wh);
        const float u = a * mxw[k] - b * (wm * m[k] - mm * c[k]);
        const float vv = u * im;
        vjp[k * nn + n] = dm;
        v[k * nn + n] = vv;
        if (vsum) vsum[k * nn + n] += vv;
    }
}

// g = vjp + M Hv (= J^T w); lam_acc += g; w_next = cl lam + cg g (or lam_out = lam_acc)
__global__ void __launch_bounds__(256)
k_adj_combine(const float *__restrict__ vjp, const float *__restrict__ Hv,
              const float *__restrict__ inv_mass, const float *__restrict__ lam,
              float *__restrict__ lam_acc, float *__restrict__ w_next, float cl, float cg,
              float *__restrict__ lam_out, int has_lin, long long nn) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * nn) return;
    const long long n = i % nn;
    const float im = inv_mass[n];
    const float M = im > 0.f ? 1.f / im : 0.f;
    const float g = vjp[i] + (has_lin ? M * Hv[i] : 0.f);
    const float acc = lam_acc[i] + g;
    if (lam_out) {
        lam_out[i] = acc;
    } else {
        lam_acc[i] = acc;
        w_next[i] = cl * lam[i] + cg * g;
    }
}

// y = a x + b z (elementwise over 3 nn)
__global__ void __launch_bounds__(256)
k_axpby(float *__restrict__ y, const float *__restrict__ x, float a, const float *__restrict__ z,
        float b, long long n3) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    y[i] = a * x[i] + (z ? b * z[i] : 0.f);
}

// grad_c += mu0 Ms_c V/8 sum_{n in c} v_n
__global__ void __launch_bounds__(256)
k_cell_gather(const float *__restrict__ v, const float *__restrict__ wc, float *__restrict__ grad,
              int N1, int N2, int N3) {
    const long long nc = (long long)N1 * N2 * N3;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    const int NX = N1 + 1, NY = N2 + 1;
    const long long nn = (long long)NX * NY * (N3 + 1);
    const int cx = (int)(c % N1), cy = (int)((c / N1) % N2), cz = (int)(c / ((long long)N1 * N2));
    for (int k = 0; k < 3; ++k) {
        float s = 0.f;
        for (int b = 0; b < 8; ++b) {
            const long long nb = ((long long)(cz + (b >> 2)) * NY + cy + ((b >> 1) & 1)) * NX + cx + (b & 1);
            s += v[k * nn + nb];
        }
        grad[k * nc + c] += wc[c] * s;
    }
}

}  // namespace nm

using namespace nm;

#define NM_REQUIRE(cond, code, msg) \
    do {                            \
        if (!(cond)) {              \
            set_error(msg);         \
            return code;            \
        }                           \
    } while (0)

#define NM_HIP(call, what)                                                          \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            set_error(std::string(what) + ": " + hipGetErrorString(e_));            \
            return NM_EHIP;                                                         \
        }                                                                           \
    } while (0)

// workspace: nsteps states + 14 nodal vectors
static long long adj_vectors(int nsteps) { return (long long)nsteps + 14; }

extern "C" size_t nm_adjoint_workspace_bytes(const nm_mesh *m, int nsteps) {
    if (!m || nsteps < 1) return 0;
    return sizeof(float) * 3 * (size_t)m->n_nodes * (size_t)adj_vectors(nsteps);
}

namespace {

hipError_t field_stage(nm_mesh *m, unsigned terms, int mode, int s, const float *in, float *out,
                       float *y_next, float *mstate, double t0, double dt) {
    if (terms & NM_T_DEMAG) {
        hipError_t e = demag_forward_conv_inverse(m, in, (terms & NM_T_ZEEMAN) ? 2 : 1);
        if (e != hipSuccess) return e;
    }
    StageSpec sp{};
    sp.mode = mode;
    sp.stage = s;
    sp.in = in;
    sp.out = out;
    sp.y_next = y_next;
    sp.mstate = mstate;
    sp.t0 = t0;
    sp.dt0 = dt;
    sp.use_ctrl = false;
    return launch_stencil(m, terms, sp);
}

}  // namespace

extern "C" nm_status nm_adjoint_step(nm_mesh *m, const float *m0, double t0, double dt, int nsteps,
                                     unsigned terms, const float *dl_dm, int dl_every, float *lambda,
                                     float *grad_hcell, float *work) {
    NM_REQUIRE(m && m0 && lambda && work, NM_EINVAL, "nm_adjoint_step: NULL argument");
    NM_REQUIRE(nsteps >= 1, NM_EINVAL, "nm_adjoint_step: nsteps must be >= 1");
    NM_REQUIRE(std::isfinite(t0) && std::isfinite(dt) && dt > 0.0, NM_EINVAL,
               "nm_adjoint_step: need finite t0 and dt > 0");
    NM_REQUIRE(!dl_dm || dl_every >= 1, NM_EINVAL, "nm_adjoint_step: dl_every must be >= 1");
    NM_REQUIRE(!(terms & ~(unsigned)NM_T_ALL), NM_EINVAL, "nm_adjoint_step: unknown term bits");
    NM_REQUIRE(!(terms & NM_T_DEMAG) || m->tensor_ready, NM_EINVAL,
               "nm_adjoint_step: NM_T_DEMAG needs nm_demag_tensor_init first");
    NM_REQUIRE(!grad_hcell || (terms & NM_T_ZEEMAN), NM_EINVAL,
               "nm_adjoint_step: a field-map gradient needs NM_T_ZEEMAN");
    const long long nn = m->n_nodes, n3 = 3 * nn;
    const size_t vb = sizeof(float) * (size_t)n3;
    float *S = work;                                   // states m_0 .. m_{nsteps-1}
    float *V = work + (long long)nsteps * n3;          // 14 scratch vectors
    float *Y[5] = {nullptr, nullptr, V + 0 * n3, V + 1 * n3, V + 2 * n3};   // y2, y3, y4
    float *Hs[5] = {nullptr, V + 3 * n3, V + 4 * n3, V + 5 * n3, V + 6 * n3};
    float *w = V + 7 * n3, *v = V + 8 * n3, *vjp = V + 9 * n3, *Hv = V + 10 * n3;
    float *lacc = V + 11 * n3, *vsum = V + 12 * n3, *wn = V + 13 * n3;
    const unsigned lin = terms & ~(unsigned)NM_T_ZEEMAN;
    const dim3 g3((unsigned)((n3 + 255) / 256)), gn((unsigned)((nn + 255) / 256));
    hipStream_t st = m->stream;
    const char *who = "nm_adjoint_step";
    const bool gather = grad_hcell != nullptr;

    // forward recompute of the segment's states from the checkpoint
    NM_HIP(hipMemcpyAsync(S, m0, vb, hipMemcpyDeviceToDevice, st), who);
    for (int j = 0; j + 1 < nsteps; ++j) {
        float *cur = S + (long long)(j + 1) * n3;
        NM_HIP(hipMemcpyAsync(cur, S + (long long)j * n3, vb, hipMemcpyDeviceToDevice, st), who);
        const double tj = t0 + j * dt;
        StageSpec sp{};
        sp.mode = kModeRK4;
        sp.t0 = tj;
        sp.dt0 = dt;
        sp.use_ctrl = false;
        sp.mstate = cur;
        const float *ins[4] = {cur, m->y[0], m->y[1], m->y[0]};
        float *outs[4] = {m->y[0], m->y[1], m->y[0], nullptr};
        for (int s = 1; s <= 4; ++s) {
            if (terms & NM_T_DEMAG)
                NM_HIP(demag_forward_conv_inverse(m, ins[s - 1], (terms & NM_T_ZEEMAN) ? 2 : 1), who);
            sp.stage = s;
            sp.in = ins[s - 1];
            sp.y_next = outs[s - 1];
            NM_HIP(launch_stencil(m, terms, sp), who);
        }
    }
    if (gather) NM_HIP(hipMemsetAsync(vsum, 0, vb, st), who);
    if (dl_dm && nsteps % dl_every == 0)
        hipLaunchKernelGGL(k_axpby, g3, dim3(256), 0, st, lambda, lambda, 1.f,
                           dl_dm + (long long)(nsteps / dl_every - 1) * n3, 1.f, n3);

    // reverse sweep
    for (int j = nsteps - 1; j >= 0; --j) {
        const double tj = t0 + j * dt;
        float *y1 = S + (long long)j * n3;
        const float *yin[5] = {nullptr, y1, Y[2], Y[3], Y[4]};
        for (int s = 1; s <= 4; ++s)
            NM_HIP(field_stage(m, terms, kModeAdjFwd, s, yin[s], Hs[s], s < 4 ? Y[s + 1] : nullptr, y1, tj, dt),
                   who);
        NM_HIP(hipMemcpyAsync(lacc, lambda, vb, hipMemcpyDeviceToDevice, st), who);
        // w4 = dt/6 lam
        hipLaunchKernelGGL(k_axpby, g3, dim3(256), 0, st, w, lambda, (float)(dt / 6.0), (const float *)nullptr,
                           0.f, n3);
        const float cl[5] = {0.f, 0.f, (float)(dt / 6.0), (float)(dt / 3.0), (float)(dt / 3.0)};
        const float cg[5] = {0.f, 0.f, (float)(dt / 2.0), (float)(dt / 2.0), (float)dt};
        for (int s = 4; s >= 1; --s) {
            hipLaunchKernelGGL(k_adj_vjp, gn, dim3(256), 0, st, yin[s], Hs[s], w, m->inv_mass, m->alpha_n,
                               m->gp_n, v, vjp, gather ? vsum : nullptr, nn);
            if (lin) {
                if (lin & NM_T_DEMAG) NM_HIP(demag_forward_conv_inverse(m, v, 1), who);
                StageSpec sp{};
                sp.mode = kModeField;
                sp.in = v;
                sp.out = Hv;
                sp.t0 = tj;
                NM_HIP(launch_stencil(m, lin, sp), who);
            }
            // s > 1: w_{s-1} = cl lam + cg J_s^T w_s; s = 1: lam <- lam_acc + J_1^T w_1
            hipLaunchKernelGGL(k_adj_combine, g3, dim3(256), 0, st, vjp, Hv, m->inv_mass, lambda, lacc, wn,
                               cl[s], cg[s], s == 1 ? lambda : nullptr, lin ? 1 : 0, nn);
            if (s > 1) std::swap(w, wn);
        }
        if (dl_dm && j > 0 && j % dl_every == 0)
            hipLaunchKernelGGL(k_axpby, g3, dim3(256), 0, st, lambda, lambda, 1.f,
                               dl_dm + (long long)(j / dl_every - 1) * n3, 1.f, n3);
    }
    if (gather)
        hipLaunchKernelGGL(k_cell_gather, dim3((unsigned)((m->n_cells + 255) / 256)), dim3(256), 0, st, vsum,
                           m->wc, grad_hcell, m->N1, m->N2, m->N3);
    NM_HIP(hipGetLastError(), who);
    return NM_OK;
}
