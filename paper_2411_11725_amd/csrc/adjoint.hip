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

// u = df/dH^T w, vjp = df/dm^T w at (y, H); v = M^-1 u, vsum += v (in
// float64: the field-map gradient sums hundreds of stage terms of both signs
// per segment, and their cancellation would amplify float32 rounding)
__global__ void __launch_bounds__(256)
k_adj_vjp(const float *__restrict__ y, const float *__restrict__ H, const float *__restrict__ w,
          const float *__restrict__ inv_mass, const float *__restrict__ alpha_n,
          const float *__restrict__ gp_n, float *__restrict__ v, float *__restrict__ vjp,
          double *__restrict__ vsum, long long nn) {
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
        if (vsum) vsum[k * nn + n] += (double)vv;
    }
}

// g = vjp + M Hv (= J^T w); lam_acc += g; w_next = cl lam + cg g (or lam_out = lam_acc).
// lam_lo: the rounding errors of the lam_acc additions (two-sums), carried
// through the segment and folded into lambda at its end, so that lambda's
// many small increments over a segment do not lose their low bits
__global__ void __launch_bounds__(256)
k_adj_combine(const float *__restrict__ vjp, const float *__restrict__ Hv,
              const float *__restrict__ inv_mass, const float *__restrict__ lam,
              float *__restrict__ lam_acc, float *__restrict__ w_next, float cl, float cg,
              float *__restrict__ lam_out, float *__restrict__ lam_lo, int has_lin, long long nn) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * nn) return;
    const long long n = i % nn;
    const float im = inv_mass[n];
    const float M = im > 0.f ? 1.f / im : 0.f;
    const float g = vjp[i] + (has_lin ? M * Hv[i] : 0.f);
    const float a = lam_acc[i];
    const float acc = a + g, bv = acc - a;
    lam_lo[i] += (a - (acc - bv)) + (g - bv);
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

// ---- continuous adjoint (Eq. adjoint_system, integrated backwards)
// At a stage state (y, a) with field H(y): f = f(y) (the LLG right-hand
// side), vjp = df/dm^T a at fixed H, v = vs M^-1 df/dH^T a; vsum += wv v
// (the field-map density, weighted by the quadrature factor).  M^-1 is of
// order 1e25 in SI units: without the scale vs (a power of two near dt) the
// linear field of v would overflow float32.
__global__ void __launch_bounds__(256)
k_cadj_node(const float *__restrict__ y, const float *__restrict__ H, const float *__restrict__ a,
            const float *__restrict__ inv_mass, const float *__restrict__ alpha_n,
            const float *__restrict__ gp_n, float *__restrict__ f, float *__restrict__ vjp,
            float *__restrict__ v, float *__restrict__ vsum, float wv, float vs, long long nn) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    if (n >= nn) return;
    float m[3], h[3], c[3];
    for (int k = 0; k < 3; ++k) {
        m[k] = y[k * nn + n];
        h[k] = H[k * nn + n];
        c[k] = a[k * nn + n];
    }
    const float ga = gp_n[n], gb = alpha_n[n] * gp_n[n], im = inv_mass[n];
    // f = -g' m x H - alpha g' m x (m x H)
    const float mxh[3] = {m[1] * h[2] - m[2] * h[1], m[2] * h[0] - m[0] * h[2], m[0] * h[1] - m[1] * h[0]};
    const float mmh[3] = {m[1] * mxh[2] - m[2] * mxh[1], m[2] * mxh[0] - m[0] * mxh[2], m[0] * mxh[1] - m[1] * mxh[0]};
    const float wm = c[0] * m[0] + c[1] * m[1] + c[2] * m[2];
    const float mh = m[0] * h[0] + m[1] * h[1] + m[2] * h[2];
    const float wh = c[0] * h[0] + c[1] * h[1] + c[2] * h[2];
    const float mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
    const float hxw[3] = {h[1] * c[2] - h[2] * c[1], h[2] * c[0] - h[0] * c[2], h[0] * c[1] - h[1] * c[0]};
    const float mxw[3] = {m[1] * c[2] - m[2] * c[1], m[2] * c[0] - m[0] * c[2], m[0] * c[1] - m[1] * c[0]};
    for (int k = 0; k < 3; ++k) {
        f[k * nn + n] = -ga * mxh[k] - gb * mmh[k];
        vjp[k * nn + n] = -ga * hxw[k] - gb * (h[k] * wm + mh * c[k] - 2.f * m[k] * wh);
        const float vv = (ga * mxw[k] - gb * (wm * m[k] - mm * c[k])) * im * vs;
        v[k * nn + n] = vv;
        if (vsum) vsum[k * nn + n] += wv * vv;
    }
}

// Clock of the continuous adjoint in the step controller: C->t_end holds the
// start of the current backward step, C->t the stage time the field kernels
// read.  op 0: start at t0; op 1: stage time = start + c h; op 2: next step.
__global__ void k_cadj_clock(Ctrl *C, int op, double t0, double ch, double h) {
    if (threadIdx.x != 0) return;
    if (op == 0) {
        C->t_end = t0;
        C->t = t0;
        C->done = 0;
    } else if (op == 1) {
        C->t = C->t_end + ch;
    } else {
        C->t_end += h;
    }
}

// Stage s of a backward RK4 step of size h on (m, a): g = -(vjp + M Hv / vs)
// is da/dt (Hv is the linear field of the scaled v); the increments are accumulated with weight b, and either the next
// stage state (m + ch f, a + ch g) is written or, after the last stage, the
// step is applied: m += h/6 (acc_m + b f), a += h/6 (acc_a + b g).
__global__ void __launch_bounds__(256)
k_cadj_combine(const float *__restrict__ f, const float *__restrict__ vjp, const float *__restrict__ Hv,
               const float *__restrict__ inv_mass, int has_lin, float inv_vs, float *__restrict__ m,
               float *__restrict__ a,
               float *__restrict__ acc_m, float *__restrict__ acc_a, float *__restrict__ ym,
               float *__restrict__ ya, float b, float ch, int first, int last, float h6, long long nn) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * nn) return;
    const long long n = i % nn;
    const float im = inv_mass[n];
    const float M = im > 0.f ? 1.f / im : 0.f;
    // (M Hv) first: M ~ 1e-26 and Hv / vs alone can exceed the float range
    const float g = -(vjp[i] + (has_lin ? (M * Hv[i]) * inv_vs : 0.f));
    const float am = (first ? 0.f : acc_m[i]) + b * f[i];
    const float aa = (first ? 0.f : acc_a[i]) + b * g;
    if (last) {
        m[i] += h6 * am;
        a[i] += h6 * aa;
    } else {
        acc_m[i] = am;
        acc_a[i] = aa;
        ym[i] = m[i] + ch * f[i];
        ya[i] = a[i] + ch * g;
    }
}

// Per-segment inputs of a recorded adjoint segment, read by the kernels of the
// graph at run time so that one graph serves every segment of the same length
struct AdjSlots {
    double t0;          // time of the segment's first state
    const float *m0;    // checkpoint state
    const float *dl;    // dL/dm samples of the segment (or NULL)
};

__global__ void k_adj_slots(AdjSlots *S, double t0, const float *m0, const float *dl) {
    if (threadIdx.x == 0) {
        S->t0 = t0;
        S->m0 = m0;
        S->dl = dl;
    }
}

// controller time of step j: t0 + j dt (read by the stage kernels)
__global__ void k_adj_time(Ctrl *C, const AdjSlots *S, int j, double dt) {
    if (threadIdx.x == 0) {
        C->t = S->t0 + j * dt;
        C->dt = dt;
        C->done = 0;
    }
}

__global__ void __launch_bounds__(256) k_vcopy(float *__restrict__ y, const float *__restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = x[i];
}

__global__ void __launch_bounds__(256) k_vadd(float *__restrict__ y, const float *__restrict__ x, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] += x[i];
}
__global__ void __launch_bounds__(256) k_vzero(float *__restrict__ y, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = 0.f;
}

__global__ void __launch_bounds__(256) k_copy_m0(float *__restrict__ y, const AdjSlots *__restrict__ S, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] = S->m0[i];
}

// y += dl[off ..]
__global__ void __launch_bounds__(256) k_add_dl(float *__restrict__ y, const AdjSlots *__restrict__ S,
                                                long long off, long long n) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i < n) y[i] += S->dl[off + i];
}

// grad_c += mu0 Ms_c V/8 sum_{n in c} v_n (the 4 nodes of a cell under the
// film basis, NZ = 1: the field map enters each of them once)
template <typename T>
__global__ void __launch_bounds__(256)
k_cell_gather(const T *__restrict__ v, const float *__restrict__ wc, float *__restrict__ grad,
              int N1, int N2, int N3, int NZ) {
    const long long nc = (long long)N1 * N2 * N3;
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    const int NX = N1 + 1, NY = N2 + 1;
    const long long nn = (long long)NX * NY * NZ;
    const int cx = (int)(c % N1), cy = (int)((c / N1) % N2), cz = (int)(c / ((long long)N1 * N2));
    for (int k = 0; k < 3; ++k) {
        T s = 0;
        for (int b = 0; b < 8; ++b) {
            if (cz + (b >> 2) >= NZ) continue;
            const long long nb = ((long long)(cz + (b >> 2)) * NY + cy + ((b >> 1) & 1)) * NX + cx + (b & 1);
            s += v[k * nn + nb];
        }
        grad[k * nc + c] += (float)(wc[c] * s);
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

// workspace: nsteps states + 15 nodal vectors, then the segment slots
static long long adj_vectors(int nsteps) { return (long long)nsteps + 18; }
static size_t adj_slot_offset(const nm_mesh *m, int nsteps) {
    const size_t b = sizeof(float) * 3 * (size_t)m->n_nodes * (size_t)adj_vectors(nsteps);
    return (b + 255) / 256 * 256;
}

extern "C" size_t nm_adjoint_workspace_bytes(const nm_mesh *m, int nsteps) {
    if (!m || nsteps < 1) return 0;
    return adj_slot_offset(m, nsteps) + 256;
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
    sp.use_ctrl = true;   // stage time from the controller (k_adj_time)
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
    NM_REQUIRE(!((terms & NM_T_CUBIC) && m->has_cubic), NM_EUNSUPPORTED,
               "nm_adjoint_step: the backward field reuses the forward one, which holds for the quadratic "
               "terms only (not the quartic cubic anisotropy)");
    const long long nn = m->n_nodes, n3 = 3 * nn;
    float *S = work;                                   // states m_0 .. m_{nsteps-1}
    float *V = work + (long long)nsteps * n3;          // 18 scratch vectors
    float *lam = V + 14 * n3;                          // lambda inside the segment
    AdjSlots *slots = reinterpret_cast<AdjSlots *>(reinterpret_cast<char *>(work) + adj_slot_offset(m, nsteps));
    const unsigned lin = terms & ~(unsigned)NM_T_ZEEMAN;
    const dim3 g3((unsigned)((n3 + 255) / 256)), gn((unsigned)((nn + 255) / 256));
    const char *who = "nm_adjoint_step";
    const bool gather = grad_hcell != nullptr;
    const bool has_dl = dl_dm != nullptr;
    // the field-map density in float64: two vectors' room from vector 15 on,
    // at an even float offset (work is 256-byte aligned; vector 17 is spare)
    float *vsum_f = V + 15 * n3 + (((long long)nsteps + 15) * n3 & 1);
    double *vsum = reinterpret_cast<double *>(vsum_f);

    // the segment body: recorded once per (length, terms, dt, loss sampling,
    // workspace) as a HIP graph and replayed for every segment; its inputs
    // (checkpoint, start time, loss samples) come through the slots
    auto enqueue = [&]() -> hipError_t {
        hipStream_t st = m->stream;
        float *Y[5] = {nullptr, nullptr, V + 0 * n3, V + 1 * n3, V + 2 * n3};   // y2, y3, y4
        float *Hs[5] = {nullptr, V + 3 * n3, V + 4 * n3, V + 5 * n3, V + 6 * n3};
        float *w = V + 7 * n3, *v = V + 8 * n3, *vjp = V + 9 * n3, *Hv = V + 10 * n3;
        float *lacc = V + 11 * n3, *wn = V + 13 * n3, *lam_lo = V + 12 * n3;
        hipError_t e = hipSuccess;
#define NM_ADJ(call)                    \
    do {                                \
        if (e == hipSuccess) e = (call); \
    } while (0)
        // forward recompute of the segment's states from the checkpoint,
        // with the compensated state update of the forward run (its carried
        // low part starts at zero at the checkpoint; the mesh's buffer is
        // borrowed, so a later RK4 call restarts its own compensation)
        hipLaunchKernelGGL(k_copy_m0, g3, dim3(256), 0, st, S, slots, n3);
        hipLaunchKernelGGL(k_vzero, g3, dim3(256), 0, st, m->mlo, n3);
        for (int j = 0; j + 1 < nsteps; ++j) {
            float *cur = S + (long long)(j + 1) * n3;
            hipLaunchKernelGGL(k_vcopy, g3, dim3(256), 0, st, cur, S + (long long)j * n3, n3);
            hipLaunchKernelGGL(k_adj_time, dim3(1), dim3(64), 0, st, m->ctrl, slots, j, dt);
            StageSpec sp{};
            sp.mode = kModeRK4;
            sp.use_ctrl = true;
            sp.mstate = cur;
            sp.lo = m->mlo;   // read by stage 4 only
            const float *ins[4] = {cur, m->y[0], m->y[1], m->y[0]};
            float *outs[4] = {m->y[0], m->y[1], m->y[0], nullptr};
            for (int s = 1; s <= 4; ++s) {
                if (terms & NM_T_DEMAG)
                    NM_ADJ(demag_forward_conv_inverse(m, ins[s - 1], (terms & NM_T_ZEEMAN) ? 2 : 1));
                sp.stage = s;
                sp.in = ins[s - 1];
                sp.y_next = outs[s - 1];
                NM_ADJ(launch_stencil(m, terms, sp));
            }
        }
        if (gather)
            hipLaunchKernelGGL(k_vzero, dim3((unsigned)((2 * n3 + 255) / 256)), dim3(256), 0, st, vsum_f, 2 * n3);
        hipLaunchKernelGGL(k_vzero, g3, dim3(256), 0, st, lam_lo, n3);
        if (has_dl && nsteps % dl_every == 0)
            hipLaunchKernelGGL(k_add_dl, g3, dim3(256), 0, st, lam, slots,
                               (long long)(nsteps / dl_every - 1) * n3, n3);
        // reverse sweep
        for (int j = nsteps - 1; j >= 0; --j) {
            float *y1 = S + (long long)j * n3;
            const float *yin[5] = {nullptr, y1, Y[2], Y[3], Y[4]};
            hipLaunchKernelGGL(k_adj_time, dim3(1), dim3(64), 0, st, m->ctrl, slots, j, dt);
            for (int s = 1; s <= 4; ++s)
                NM_ADJ(field_stage(m, terms, kModeAdjFwd, s, yin[s], Hs[s], s < 4 ? Y[s + 1] : nullptr, y1, 0.0,
                                   dt));
            hipLaunchKernelGGL(k_vcopy, g3, dim3(256), 0, st, lacc, lam, n3);
            // w4 = dt/6 lam
            hipLaunchKernelGGL(k_axpby, g3, dim3(256), 0, st, w, lam, (float)(dt / 6.0), (const float *)nullptr,
                               0.f, n3);
            const float cl[5] = {0.f, 0.f, (float)(dt / 6.0), (float)(dt / 3.0), (float)(dt / 3.0)};
            const float cg[5] = {0.f, 0.f, (float)(dt / 2.0), (float)(dt / 2.0), (float)dt};
            for (int s = 4; s >= 1; --s) {
                hipLaunchKernelGGL(k_adj_vjp, gn, dim3(256), 0, st, yin[s], Hs[s], w, m->inv_mass, m->alpha_n,
                                   m->gp_n, v, vjp, gather ? vsum : nullptr, nn);
                if (lin) {
                    if (lin & NM_T_DEMAG) NM_ADJ(demag_forward_conv_inverse(m, v, 1));
                    StageSpec sp{};
                    sp.mode = kModeField;
                    sp.in = v;
                    sp.out = Hv;
                    NM_ADJ(launch_stencil(m, lin, sp));
                }
                // s > 1: w_{s-1} = cl lam + cg J_s^T w_s; s = 1: lam <- lam_acc + J_1^T w_1
                hipLaunchKernelGGL(k_adj_combine, g3, dim3(256), 0, st, vjp, Hv, m->inv_mass, lam, lacc, wn,
                                   cl[s], cg[s], s == 1 ? lam : nullptr, lam_lo, lin ? 1 : 0, nn);
                if (s > 1) std::swap(w, wn);
            }
            if (has_dl && j > 0 && j % dl_every == 0)
                hipLaunchKernelGGL(k_add_dl, g3, dim3(256), 0, st, lam, slots, (long long)(j / dl_every - 1) * n3,
                                   n3);
        }
        hipLaunchKernelGGL(k_vadd, g3, dim3(256), 0, st, lam, lam_lo, n3);   // fold the low part in
#undef NM_ADJ
        return e == hipSuccess ? hipGetLastError() : e;
    };

    hipStream_t st = m->stream;
    hipLaunchKernelGGL(k_adj_slots, dim3(1), dim3(64), 0, st, slots, t0, m0, dl_dm);
    hipLaunchKernelGGL(k_vcopy, g3, dim3(256), 0, st, lam, lambda, n3);
    if (m->prof) {
        NM_HIP(enqueue(), who);   // per-kernel events cannot live in a graph
    } else {
        const bool same = m->adj_gexec && m->adj_nsteps == nsteps && m->adj_terms == terms && m->adj_dt == dt &&
                          m->adj_every == (has_dl ? dl_every : 0) && m->adj_gather == gather &&
                          m->adj_work == work;
        if (!same) {
            if (m->adj_gexec) {
                (void)hipStreamSynchronize(st);
                (void)hipGraphExecDestroy(m->adj_gexec);
                m->adj_gexec = nullptr;
            }
            m->stream = m->cap_stream;
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed);
            hipError_t e2 = e == hipSuccess ? enqueue() : e;
            if (e == hipSuccess) e = hipStreamEndCapture(m->cap_stream, &graph);
            m->stream = st;
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&m->adj_gexec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            NM_HIP(e, who);
            m->adj_nsteps = nsteps;
            m->adj_terms = terms;
            m->adj_dt = dt;
            m->adj_every = has_dl ? dl_every : 0;
            m->adj_gather = gather;
            m->adj_work = work;
        }
        NM_HIP(hipGraphLaunch(m->adj_gexec, st), who);
    }
    hipLaunchKernelGGL(k_vcopy, g3, dim3(256), 0, st, lambda, lam, n3);
    if (gather)
        hipLaunchKernelGGL(k_cell_gather<double>, dim3((unsigned)((m->n_cells + 255) / 256)), dim3(256), 0, st,
                           (const double *)vsum, m->wc, grad_hcell, m->N1, m->N2, m->N3, m->NZ);
    NM_HIP(hipGetLastError(), who);
    m->lo_valid = false;   // the recompute used the RK4 compensation buffer
    return NM_OK;
}

// The adjoint system of Sec. 4 integrated backwards: classical RK4 steps of
// h = -dt on (m, a, u), one recorded graph replayed per step.  Per stage the field H(y) gives f and the node-local
// part of (df/dm)^T a; the transpose of the linear field is the forward
// linear field of v = M^-1 (df/dH)^T a (as in the discrete adjoint), and the
// field-map density v is accumulated with the weight -h/6 b_s of u's
// quadrature, then gathered to cells once.  The mesh's stepping buffers
// hold the stage vectors, so no trajectory is stored.
extern "C" nm_status nm_adjoint_continuous(nm_mesh *m, float *mag, double t_end, double dt, int nsteps,
                                           unsigned terms, float *a, float *grad_hcell) {
    const char *who = "nm_adjoint_continuous";
    NM_REQUIRE(m && mag && a, NM_EINVAL, "nm_adjoint_continuous: NULL argument");
    NM_REQUIRE(nsteps >= 1, NM_EINVAL, "nm_adjoint_continuous: nsteps must be >= 1");
    NM_REQUIRE(std::isfinite(t_end) && std::isfinite(dt) && dt > 0.0, NM_EINVAL,
               "nm_adjoint_continuous: need finite t_end and dt > 0");
    NM_REQUIRE(!(terms & ~(unsigned)NM_T_ALL), NM_EINVAL, "nm_adjoint_continuous: unknown term bits");
    NM_REQUIRE(!(terms & NM_T_DEMAG) || m->tensor_ready, NM_EINVAL,
               "nm_adjoint_continuous: NM_T_DEMAG needs nm_demag_tensor_init first");
    NM_REQUIRE(!grad_hcell || (terms & NM_T_ZEEMAN), NM_EINVAL,
               "nm_adjoint_continuous: a field-map gradient needs NM_T_ZEEMAN");
    NM_REQUIRE(!((terms & NM_T_CUBIC) && m->has_cubic), NM_EUNSUPPORTED,
               "nm_adjoint_continuous: the backward field reuses the forward one, which holds for the quadratic "
               "terms only (not the quartic cubic anisotropy)");
    const long long nn = m->n_nodes, n3 = 3 * nn;
    const dim3 g3((unsigned)((n3 + 255) / 256)), gn((unsigned)((nn + 255) / 256));
    hipStream_t st = m->stream;
    float *ym = m->y[0], *ya = m->y[1], *H = m->acc, *f = m->k[0], *vjp = m->k[1], *v = m->k[2];
    float *Hv = m->k[3], *accm = m->k[4], *acca = m->k[5], *vsum = m->k[6];
    const unsigned lin = terms & ~(unsigned)NM_T_ZEEMAN;
    const bool gather = grad_hcell != nullptr;
    const double h = -dt;
    const double c[4] = {0.0, 0.5, 0.5, 1.0}, b[4] = {1.0, 2.0, 2.0, 1.0};
    // v is scaled by a power of two near dt (exact in float32), as the
    // discrete adjoint's co-vectors carry dt
    const double vs = std::ldexp(1.0, (int)std::floor(std::log2(dt)));
    if (gather) hipLaunchKernelGGL(k_vzero, g3, dim3(256), 0, st, vsum, n3);
    hipLaunchKernelGGL(k_cadj_clock, dim3(1), dim3(64), 0, st, m->ctrl, 0, t_end, 0.0, 0.0);
    // one backward step; its stage times come from the controller, so one
    // recorded graph serves every step
    auto enqueue = [&]() -> hipError_t {
        hipStream_t s0 = m->stream;
        hipError_t e = hipSuccess;
        for (int s = 0; s < 4 && e == hipSuccess; ++s) {
            const float *yin = s == 0 ? mag : ym;
            const float *ain = s == 0 ? a : ya;
            hipLaunchKernelGGL(k_cadj_clock, dim3(1), dim3(64), 0, s0, m->ctrl, 1, 0.0, c[s] * h, 0.0);
            // H at the stage state and time
            if (terms & NM_T_DEMAG) e = demag_forward_conv_inverse(m, yin, (terms & NM_T_ZEEMAN) ? 2 : 1);
            StageSpec sp{};
            sp.mode = kModeField;
            sp.in = yin;
            sp.out = H;
            sp.use_ctrl = true;
            if (e == hipSuccess) e = launch_stencil(m, terms, sp);
            hipLaunchKernelGGL(k_cadj_node, gn, dim3(256), 0, s0, yin, H, ain, m->inv_mass, m->alpha_n, m->gp_n,
                               f, vjp, v, gather ? vsum : nullptr, (float)(-h / 6.0 * b[s] / vs), (float)vs, nn);
            if (lin) {
                if ((lin & NM_T_DEMAG) && e == hipSuccess) e = demag_forward_conv_inverse(m, v, 1);
                StageSpec sl{};
                sl.mode = kModeField;
                sl.in = v;
                sl.out = Hv;
                if (e == hipSuccess) e = launch_stencil(m, lin, sl);
            }
            hipLaunchKernelGGL(k_cadj_combine, g3, dim3(256), 0, s0, f, vjp, Hv, m->inv_mass, lin ? 1 : 0,
                               (float)(1.0 / vs), mag, a, accm, acca, ym, ya, (float)b[s],
                               (float)((s < 3 ? c[s + 1] : 0.0) * h), s == 0 ? 1 : 0, s == 3 ? 1 : 0,
                               (float)(h / 6.0), nn);
        }
        hipLaunchKernelGGL(k_cadj_clock, dim3(1), dim3(64), 0, s0, m->ctrl, 2, 0.0, 0.0, h);
        return e == hipSuccess ? hipGetLastError() : e;
    };
    if (m->prof) {
        for (int j = 0; j < nsteps; ++j) NM_HIP(enqueue(), who);   // per-kernel events: direct launches
    } else {
        const bool same = m->cadj_gexec && m->cadj_terms == terms && m->cadj_dt == dt &&
                          m->cadj_gather == gather && m->cadj_m == mag && m->cadj_a == a;
        if (!same) {
            if (m->cadj_gexec) {
                (void)hipStreamSynchronize(st);
                (void)hipGraphExecDestroy(m->cadj_gexec);
                m->cadj_gexec = nullptr;
            }
            m->stream = m->cap_stream;
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed);
            hipError_t e2 = e == hipSuccess ? enqueue() : e;
            if (e == hipSuccess) e = hipStreamEndCapture(m->cap_stream, &graph);
            m->stream = st;
            if (e == hipSuccess) e = e2;
            if (e == hipSuccess) e = hipGraphInstantiate(&m->cadj_gexec, graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            NM_HIP(e, who);
            m->cadj_terms = terms;
            m->cadj_dt = dt;
            m->cadj_gather = gather;
            m->cadj_m = mag;
            m->cadj_a = a;
        }
        for (int j = 0; j < nsteps; ++j) NM_HIP(hipGraphLaunch(m->cadj_gexec, st), who);
    }
    if (gather)
        hipLaunchKernelGGL(k_cell_gather<float>, dim3((unsigned)((m->n_cells + 255) / 256)), dim3(256), 0, st, vsum,
                           m->wc, grad_hcell, m->N1, m->N2, m->N3, m->NZ);
    NM_HIP(hipGetLastError(), who);
    return NM_OK;
}
