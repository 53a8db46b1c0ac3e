// Local field terms, LLG right-hand side and Runge-Kutta stage epilogues,
// fused node by node (gfx950).
//
// For node n the variation dE/dm_n is gathered from the (up to) 8 cells that
// share it (Eqs. weak_form_impl_f and weak_form_impl, evaluated per node
// instead of scattered per cell, so no atomics are needed):
//   exchange    2 A_c sum_b K^e_ab (m_b - m_n)     (K^e rows sum to zero, so
//               the differences keep float32 accurate near uniform states)
//   anisotropy  -2 Ku_c e_c sum_b M^e_ab (m_b . e_c)
//   cell fields -mu0 Ms_c V/8 H_c  (Zeeman and the demag cell field)
// with a = local index of n in cell c.  K^e and M^e of a cuboid cell depend
// only on which axes a and b differ in, so 8 numbers each describe them.
// Mass lumping (Eq. mass_lumping) then gives H_n = -g_n / M_n, and the LLG
// right-hand side (Eq. llg) is evaluated in the same thread.
#include <cmath>

#include "nm_internal.h"

namespace nm {

struct StencilParams {
    int N1, N2, N3, NX, NY, NZ;
    long long nn, nc;
    float Kp[8], Mp[8];
    const float *wc, *A2, *Ku, *easy, *hcell, *dmask, *hd;
    float hu[3], damp[3];
    double dfreq, dphase;
    const float *inv_mass, *alpha_n, *gp_n;
    unsigned terms;
};

struct StageArgs {
    const float *in;
    float *out, *y_next, *mstate, *acc;
    float *k[7];
    const Ctrl *ctrl;
    ErrPartial *partials;
    double t0, c;
    double a[7], e[7];
    int stage;
};

__device__ __forceinline__ void node_field(const StencilParams &P, const float *__restrict__ m,
                                           long long n, double t, float mn[3], float H[3]) {
    const int x = (int)(n % P.NX);
    const long long r = n / P.NX;
    const int y = (int)(r % P.NY);
    const int z = (int)(r / P.NY);
    const long long nn = P.nn, nc = P.nc;
    mn[0] = m[n];
    mn[1] = m[nn + n];
    mn[2] = m[2 * nn + n];
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;   // dE/dm of exchange + anisotropy
    float s0 = 0.f, s1 = 0.f, s2 = 0.f;   // sum_c mu0 Ms_c V/8 (H_ext + H_d)_c
    const bool ex = P.terms & NM_T_EXCHANGE;
    const bool an = (P.terms & NM_T_ANIS) && P.Ku;
    const bool ze = P.terms & NM_T_ZEEMAN;
    const bool dm = (P.terms & NM_T_DEMAG) && P.hd;
    float sdrive = 0.f;
    if (ze && P.dmask) sdrive = (float)sin(2.0 * 3.14159265358979323846 * P.dfreq * t + P.dphase);
#pragma unroll
    for (int i3 = 0; i3 < 2; ++i3) {
        const int cz = z - i3;
        if (cz < 0 || cz >= P.N3) continue;
#pragma unroll
        for (int i2 = 0; i2 < 2; ++i2) {
            const int cy = y - i2;
            if (cy < 0 || cy >= P.N2) continue;
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1) {
                const int cx = x - i1;
                if (cx < 0 || cx >= P.N1) continue;
                const long long c = ((long long)cz * P.N2 + cy) * P.N1 + cx;
                if (ex || an) {
                    const float a2 = ex ? P.A2[c] : 0.f;
                    float e0 = 0.f, e1 = 0.f, e2 = 0.f, ku = 0.f, sp = 0.f;
                    if (an) {
                        ku = P.Ku[c];
                        e0 = P.easy[c];
                        e1 = P.easy[nc + c];
                        e2 = P.easy[2 * nc + c];
                    }
#pragma unroll
                    for (int b3 = 0; b3 < 2; ++b3)
#pragma unroll
                        for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
                            for (int b1 = 0; b1 < 2; ++b1) {
                                const int mask = (i1 ^ b1) | ((i2 ^ b2) << 1) | ((i3 ^ b3) << 2);
                                float v0, v1, v2;
                                if (mask == 0) {
                                    v0 = mn[0];
                                    v1 = mn[1];
                                    v2 = mn[2];
                                } else {
                                    const long long nb = ((long long)(cz + b3) * P.NY + (cy + b2)) * P.NX + (cx + b1);
                                    v0 = m[nb];
                                    v1 = m[nn + nb];
                                    v2 = m[2 * nn + nb];
                                    if (ex) {
                                        const float w = a2 * P.Kp[mask];
                                        g0 += w * (v0 - mn[0]);
                                        g1 += w * (v1 - mn[1]);
                                        g2 += w * (v2 - mn[2]);
                                    }
                                }
                                if (an) sp += P.Mp[mask] * (v0 * e0 + v1 * e1 + v2 * e2);
                            }
                    if (an) {
                        const float k2 = -2.f * ku * sp;
                        g0 += k2 * e0;
                        g1 += k2 * e1;
                        g2 += k2 * e2;
                    }
                }
                if (ze || dm) {
                    const float w = P.wc[c];
                    float h0 = 0.f, h1 = 0.f, h2 = 0.f;
                    if (ze) {
                        h0 = P.hu[0];
                        h1 = P.hu[1];
                        h2 = P.hu[2];
                        if (P.hcell) {
                            h0 += P.hcell[c];
                            h1 += P.hcell[nc + c];
                            h2 += P.hcell[2 * nc + c];
                        }
                        if (P.dmask) {
                            const float d = P.dmask[c] * sdrive;
                            h0 += d * P.damp[0];
                            h1 += d * P.damp[1];
                            h2 += d * P.damp[2];
                        }
                    }
                    if (dm) {
                        h0 += P.hd[c];
                        h1 += P.hd[nc + c];
                        h2 += P.hd[2 * nc + c];
                    }
                    s0 += w * h0;
                    s1 += w * h1;
                    s2 += w * h2;
                }
            }
        }
    }
    const float im = P.inv_mass[n];
    H[0] = (s0 - g0) * im;
    H[1] = (s1 - g1) * im;
    H[2] = (s2 - g2) * im;
}

__device__ __forceinline__ void llg_rhs(const float m[3], const float H[3], float gp, float al,
                                        float f[3]) {
    const float c0 = m[1] * H[2] - m[2] * H[1];
    const float c1 = m[2] * H[0] - m[0] * H[2];
    const float c2 = m[0] * H[1] - m[1] * H[0];
    const float d0 = m[1] * c2 - m[2] * c1;
    const float d1 = m[2] * c0 - m[0] * c2;
    const float d2 = m[0] * c1 - m[1] * c0;
    const float ag = al * gp;
    f[0] = -gp * c0 - ag * d0;
    f[1] = -gp * c1 - ag * d1;
    f[2] = -gp * c2 - ag * d2;
}

// block reduction of the DP45 error partials (256 threads = 4 waves)
__device__ __forceinline__ void reduce_partial(double sq, float mf, int nf, ErrPartial *out) {
    __shared__ double s_sq[256];
    __shared__ float s_mf[256];
    __shared__ int s_nf[256];
    const int t = threadIdx.x;
    s_sq[t] = sq;
    s_mf[t] = mf;
    s_nf[t] = nf;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s_sq[t] += s_sq[t + w];
            s_mf[t] = fmaxf(s_mf[t], s_mf[t + w]);
            s_nf[t] |= s_nf[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[blockIdx.x].sumsq = s_sq[0];
        out[blockIdx.x].maxf = s_mf[0];
        out[blockIdx.x].nonfinite = s_nf[0];
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_stencil(StencilParams P, StageArgs S) {
    const long long n = (long long)blockIdx.x * 256 + threadIdx.x;
    double t = S.t0, dt = 0.0;
    const Ctrl *C = S.ctrl;
    if (C) {
        if (C->done) return;
        dt = C->dt;
        t = C->t + S.c * dt;
    }
    const long long nn = P.nn;
    const bool valid = n < nn;
    float mn[3] = {0.f, 0.f, 0.f}, H[3] = {0.f, 0.f, 0.f}, f[3] = {0.f, 0.f, 0.f};
    if (valid) {
        node_field(P, S.in, n, t, mn, H);
        if (MODE != kModeField) llg_rhs(mn, H, P.gp_n[n], P.alpha_n[n], f);
    }
    if (MODE == kModeField) {
        if (valid)
            for (int c = 0; c < 3; ++c) S.out[c * nn + n] = H[c];
    } else if (MODE == kModeRhs) {
        if (valid)
            for (int c = 0; c < 3; ++c) S.out[c * nn + n] = f[c];
    } else if (MODE == kModeRK4) {
        if (!valid) return;
        const int s = S.stage;
        const float wacc = s == 1 ? 1.f : 2.f;
        const float cy = (float)(dt * (s == 3 ? 1.0 : 0.5));
        const float c6 = (float)(dt / 6.0);
        for (int c = 0; c < 3; ++c) {
            const long long i = c * nn + n;
            const float ms = S.mstate[i];
            if (s == 4) {
                S.mstate[i] = ms + c6 * (S.acc[i] + f[c]);
            } else {
                S.acc[i] = s == 1 ? f[c] : S.acc[i] + wacc * f[c];
                S.y_next[i] = ms + cy * f[c];
            }
        }
    } else {  // DP45 stage s: store k_s, form y_{s+1}, or the error norm at s = 7
        const int s = S.stage;
        double sq = 0.0;
        float mf = 0.f;
        int nf = 0;
        if (valid) {
            const bool active = P.inv_mass[n] > 0.f;
            float a[7];
            for (int j = 0; j < 7; ++j) a[j] = (float)(dt * (s < 7 ? S.a[j] : S.e[j]));
            float fn2 = 0.f;
            for (int c = 0; c < 3; ++c) {
                const long long i = c * nn + n;
                S.k[s - 1][i] = f[c];
                float acc = a[s - 1] * f[c];
                for (int j = 0; j < s - 1; ++j)
                    if (a[j] != 0.f) acc += a[j] * S.k[j][i];
                const float ms = S.mstate[i];
                if (s < 7) {
                    S.y_next[i] = ms + acc;
                } else {
                    const float yn = S.in[i];
                    const double sc = C->atol + C->rtol * fmax(fabs((double)ms), fabs((double)yn));
                    const double r = (double)acc / sc;
                    if (active) sq += r * r;
                    if (!isfinite(acc) || !isfinite(yn)) nf = 1;
                    fn2 += f[c] * f[c];
                }
            }
            if (s == 7 && active) mf = sqrtf(fn2);
        }
        if (s == 7) reduce_partial(sq, mf, nf, S.partials);
    }
}

// ---------------------------------------------------------------- energies
__global__ void __launch_bounds__(256) k_energy_cells(StencilParams P, const float *__restrict__ m,
                                                      double t, double *__restrict__ part) {
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    float eex = 0.f, ean = 0.f, ez = 0.f, ed = 0.f;
    if (c < P.nc) {
        const int cx = (int)(c % P.N1);
        const long long r = c / P.N1;
        const int cy = (int)(r % P.N2);
        const int cz = (int)(r / P.N2);
        float v[8][3];
        for (int b = 0; b < 8; ++b) {
            const long long nb = ((long long)(cz + (b >> 2)) * P.NY + (cy + ((b >> 1) & 1))) * P.NX + cx + (b & 1);
            for (int k = 0; k < 3; ++k) v[b][k] = m[k * P.nn + nb];
        }
        if (P.terms & NM_T_EXCHANGE) {
            // m^T K m = -sum_{a<b} K_ab |m_a - m_b|^2 (rows of K sum to zero)
            float s = 0.f;
            for (int a = 0; a < 8; ++a)
                for (int b = a + 1; b < 8; ++b) {
                    const float d0 = v[a][0] - v[b][0], d1 = v[a][1] - v[b][1], d2 = v[a][2] - v[b][2];
                    s += P.Kp[a ^ b] * (d0 * d0 + d1 * d1 + d2 * d2);
                }
            eex = -0.5f * P.A2[c] * s;
        }
        if ((P.terms & NM_T_ANIS) && P.Ku) {
            const float e0 = P.easy[c], e1 = P.easy[P.nc + c], e2 = P.easy[2 * P.nc + c];
            float p[8];
            for (int b = 0; b < 8; ++b) p[b] = v[b][0] * e0 + v[b][1] * e1 + v[b][2] * e2;
            float s = 0.f;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) s += P.Mp[a ^ b] * p[a] * p[b];
            ean = -P.Ku[c] * s;
        }
        float ms0 = 0.f, ms1 = 0.f, ms2 = 0.f;
        for (int b = 0; b < 8; ++b) {
            ms0 += v[b][0];
            ms1 += v[b][1];
            ms2 += v[b][2];
        }
        const float w = P.wc[c];
        if (P.terms & NM_T_ZEEMAN) {
            float h0 = P.hu[0], h1 = P.hu[1], h2 = P.hu[2];
            if (P.hcell) {
                h0 += P.hcell[c];
                h1 += P.hcell[P.nc + c];
                h2 += P.hcell[2 * P.nc + c];
            }
            if (P.dmask) {
                const float d = P.dmask[c] * (float)sin(2.0 * 3.14159265358979323846 * P.dfreq * t + P.dphase);
                h0 += d * P.damp[0];
                h1 += d * P.damp[1];
                h2 += d * P.damp[2];
            }
            ez = -w * (ms0 * h0 + ms1 * h1 + ms2 * h2);
        }
        if ((P.terms & NM_T_DEMAG) && P.hd)
            ed = -0.5f * w * (ms0 * P.hd[c] + ms1 * P.hd[P.nc + c] + ms2 * P.hd[2 * P.nc + c]);
    }
    __shared__ double s[4][256];
    const int t0 = threadIdx.x;
    s[0][t0] = eex;
    s[1][t0] = ed;
    s[2][t0] = ean;
    s[3][t0] = ez;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t0 < w)
            for (int k = 0; k < 4; ++k) s[k][t0] += s[k][t0 + w];
        __syncthreads();
    }
    if (t0 < 4) part[(long long)t0 * gridDim.x + blockIdx.x] = s[t0][0];
}

__global__ void k_energy_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double s[256];
    for (int k = 0; k < 4; ++k) {
        double acc = 0.0;
        for (int i = threadIdx.x; i < nb; i += 256) acc += part[(long long)k * nb + i];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = s[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------- step control
__global__ void k_dp45_control(Ctrl *C, const ErrPartial *__restrict__ part, int np) {
    __shared__ double s_sq[256];
    __shared__ float s_mf[256];
    __shared__ int s_nf[256];
    if (C->done) {
        if (threadIdx.x == 0) C->accept = 0;
        return;
    }
    double sq = 0.0;
    float mf = 0.f;
    int nf = 0;
    for (int i = threadIdx.x; i < np; i += 256) {
        sq += part[i].sumsq;
        mf = fmaxf(mf, part[i].maxf);
        nf |= part[i].nonfinite;
    }
    const int t = threadIdx.x;
    s_sq[t] = sq;
    s_mf[t] = mf;
    s_nf[t] = nf;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s_sq[t] += s_sq[t + w];
            s_mf[t] = fmaxf(s_mf[t], s_mf[t + w]);
            s_nf[t] |= s_nf[t + w];
        }
        __syncthreads();
    }
    if (t != 0) return;
    const double err = sqrt(s_sq[0] * C->norm_scale);
    C->accept = 0;
    C->err = err;
    C->rhs_evals += 6;
    if (s_nf[0] || !isfinite(err)) {
        C->status = NM_ENONFINITE;
        C->done = 1;
        return;
    }
    double fac = err == 0.0 ? 5.0 : fmin(5.0, fmax(0.2, 0.9 * pow(err, -0.2)));
    const bool last = C->dt >= (C->t_end - C->t) * (1.0 - 1e-9);
    if (C->log && C->attempts < C->log_cap) {
        double *L = C->log + 3 * C->attempts;
        L[0] = C->t;
        L[1] = C->dt;
        L[2] = err <= 1.0 ? 1.0 : 0.0;
    }
    C->attempts += 1;
    if (err <= 1.0) {
        C->accept = 1;
        C->accepted += 1;
        C->t = last ? C->t_end : C->t + C->dt;
        C->max_torque = s_mf[0];
        if (C->rejected_last) fac = fmin(fac, 1.0);
        C->rejected_last = 0;
        if (last || (C->stop_torque > 0.0 && s_mf[0] < C->stop_torque) || C->accepted >= C->max_accepted)
            C->done = 1;
    } else {
        C->rejected += 1;
        C->rejected_last = 1;
    }
    double dtn = C->dt * fac;
    if (C->dt_max > 0.0) dtn = fmin(dtn, C->dt_max);
    C->dt_prop = dtn;
    if (!C->done && dtn < C->dt_min) {
        C->status = NM_ESTEPSIZE;
        C->done = 1;
    }
    C->dt = fmin(dtn, C->t_end - C->t);
}

__global__ void k_dp45_finish(const Ctrl *__restrict__ C, float *__restrict__ mstate,
                              const float *__restrict__ y7, float *__restrict__ k1,
                              const float *__restrict__ k7, float *__restrict__ y2, long long n3,
                              double a21) {
    const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n3) return;
    const bool acc = C->accept;
    const bool done = C->done;
    if (!acc && done) return;
    float mv = mstate[i], kv = k1[i];
    if (acc) {
        mv = y7[i];
        kv = k7[i];
        mstate[i] = mv;
        k1[i] = kv;
    }
    if (!done) y2[i] = mv + (float)(C->dt * a21) * kv;
}

__global__ void k_rk4_advance(Ctrl *C) {
    if (C->done) return;
    const bool last = C->dt >= (C->t_end - C->t) * (1.0 - 1e-9);
    C->t = last ? C->t_end : C->t + C->dt;
    C->accepted += 1;
    C->attempts += 1;
    C->rhs_evals += 4;
    if (last || C->accepted >= C->max_accepted) C->done = 1;
    else C->dt = fmin(C->dt_prop, C->t_end - C->t);
}

// ------------------------------------------------------------- launchers
static StencilParams make_params(const nm_mesh *m, unsigned terms) {
    StencilParams P;
    P.N1 = m->N1;
    P.N2 = m->N2;
    P.N3 = m->N3;
    P.NX = m->NX;
    P.NY = m->NY;
    P.NZ = m->NZ;
    P.nn = m->n_nodes;
    P.nc = m->n_cells;
    for (int i = 0; i < 8; ++i) {
        P.Kp[i] = m->Kp[i];
        P.Mp[i] = m->Mp[i];
    }
    P.wc = m->wc;
    P.A2 = m->A2;
    P.Ku = m->has_anis ? m->Ku : nullptr;
    P.easy = m->has_anis ? m->easy : nullptr;
    P.hcell = m->has_hcell ? m->h_cell : nullptr;
    P.dmask = m->has_drive ? m->drive_mask : nullptr;
    P.hd = (terms & NM_T_DEMAG) ? m->hd : nullptr;
    for (int i = 0; i < 3; ++i) {
        P.hu[i] = m->h_uniform[i];
        P.damp[i] = m->drive_amp[i];
    }
    P.dfreq = m->drive_freq;
    P.dphase = m->drive_phase;
    P.inv_mass = m->inv_mass;
    P.alpha_n = m->alpha_n;
    P.gp_n = m->gp_n;
    P.terms = terms;
    return P;
}

hipError_t launch_stencil(nm_mesh *m, unsigned terms, const StageSpec &sp) {
    StencilParams P = make_params(m, terms);
    StageArgs S{};
    S.in = sp.in;
    S.out = sp.out;
    S.y_next = sp.y_next;
    S.t0 = sp.t0;
    S.c = sp.c;
    S.stage = sp.stage;
    S.ctrl = sp.use_ctrl ? m->ctrl : nullptr;
    S.partials = m->partials;
    for (int j = 0; j < 7; ++j) {
        S.a[j] = sp.a[j];
        S.e[j] = sp.e[j];
        S.k[j] = m->k[j];
    }
    S.acc = m->acc;
    S.mstate = sp.mstate;
    const unsigned grid = (unsigned)((m->n_nodes + 255) / 256);
    ProfScope ps(m, NM_PROF_STENCIL);
    switch (sp.mode) {
        case kModeField:
            hipLaunchKernelGGL((k_stencil<kModeField>), dim3(grid), dim3(256), 0, m->stream, P, S);
            break;
        case kModeRhs:
            hipLaunchKernelGGL((k_stencil<kModeRhs>), dim3(grid), dim3(256), 0, m->stream, P, S);
            break;
        case kModeRK4:
            hipLaunchKernelGGL((k_stencil<kModeRK4>), dim3(grid), dim3(256), 0, m->stream, P, S);
            break;
        default:
            hipLaunchKernelGGL((k_stencil<kModeDP45>), dim3(grid), dim3(256), 0, m->stream, P, S);
            break;
    }
    return hipGetLastError();
}

hipError_t launch_energy(nm_mesh *m, const float *mag, unsigned terms, double t, double e[5]) {
    StencilParams P = make_params(m, terms);
    const unsigned grid = (unsigned)((m->n_cells + 255) / 256);
    if ((int)grid > m->n_eblocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_cells, dim3(grid), dim3(256), 0, m->stream, P, mag, t, m->ered);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, m->stream, m->ered, (int)grid,
                       m->ered + 4LL * m->n_eblocks);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    double host[4];
    err = hipMemcpyAsync(host, m->ered + 4LL * m->n_eblocks, sizeof(host), hipMemcpyDeviceToHost,
                         m->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(m->stream);
    if (err != hipSuccess) return err;
    for (int k = 0; k < 4; ++k) e[k] = host[k];
    e[4] = host[0] + host[1] + host[2] + host[3];
    return hipSuccess;
}

hipError_t launch_dp45_control(nm_mesh *m) {
    const int np = (int)((m->n_nodes + 255) / 256);
    ProfScope ps(m, NM_PROF_CONTROL);
    hipLaunchKernelGGL(k_dp45_control, dim3(1), dim3(256), 0, m->stream, m->ctrl, m->partials, np);
    return hipGetLastError();
}

hipError_t launch_dp45_finish(nm_mesh *m, float *mstate, double a21) {
    const long long n3 = 3 * m->n_nodes;
    ProfScope ps(m, NM_PROF_CONTROL);
    hipLaunchKernelGGL(k_dp45_finish, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, m->stream,
                       m->ctrl, mstate, m->y[1], m->k[0], m->k[6], m->y[0], n3, a21);
    return hipGetLastError();
}

hipError_t launch_rk4_advance(nm_mesh *m) {
    ProfScope ps(m, NM_PROF_CONTROL);
    hipLaunchKernelGGL(k_rk4_advance, dim3(1), dim3(1), 0, m->stream, m->ctrl);
    return hipGetLastError();
}

}  // namespace nm
