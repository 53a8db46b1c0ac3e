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
//   interfacial DMI (antisymmetric exchange, Sec. 2)
//               D_c sum_b (-A_x m_b,z, -A_y m_b,z, A_x m_b,x + A_y m_b,y)_ab
// with a = local index of n in cell c.  K^e and M^e of a cuboid cell depend
// only on which axes a and b differ in, so 8 numbers each describe them.
// Mass lumping (Eq. mass_lumping) then gives H_n = -g_n / M_n, and the LLG
// right-hand side (Eq. llg) is evaluated in the same thread.
#include <cmath>

#include "nm_internal.h"

namespace nm {

// Dormand & Prince (1980) RK5(4)7FM: y_{s+1} = m + dt sum_{j<=s} a_{s+1,j} k_j
__host__ __device__ constexpr double dp_c(int s) {  // stage s (1-based) time fraction
    return s == 1 ? 0.0 : s == 2 ? 1.0 / 5 : s == 3 ? 3.0 / 10 : s == 4 ? 4.0 / 5 : s == 5 ? 8.0 / 9 : 1.0;
}
__host__ __device__ constexpr double dp_a(int r, int j) {  // a_{r,j}, 1-based
    return r == 2 ? (j == 1 ? 1.0 / 5 : 0.0)
         : r == 3 ? (j == 1 ? 3.0 / 40 : j == 2 ? 9.0 / 40 : 0.0)
         : r == 4 ? (j == 1 ? 44.0 / 45 : j == 2 ? -56.0 / 15 : j == 3 ? 32.0 / 9 : 0.0)
         : r == 5 ? (j == 1 ? 19372.0 / 6561 : j == 2 ? -25360.0 / 2187 : j == 3 ? 64448.0 / 6561
                     : j == 4 ? -212.0 / 729 : 0.0)
         : r == 6 ? (j == 1 ? 9017.0 / 3168 : j == 2 ? -355.0 / 33 : j == 3 ? 46732.0 / 5247
                     : j == 4 ? 49.0 / 176 : j == 5 ? -5103.0 / 18656 : 0.0)
         : r == 7 ? (j == 1 ? 35.0 / 384 : j == 2 ? 0.0 : j == 3 ? 500.0 / 1113 : j == 4 ? 125.0 / 192
                     : j == 5 ? -2187.0 / 6784 : j == 6 ? 11.0 / 84 : 0.0)
         : 0.0;
}
// embedded error weights b_j - b*_j
__host__ __device__ constexpr double dp_e(int j) {
    return j == 1 ? 35.0 / 384 - 5179.0 / 57600 : j == 2 ? 0.0 : j == 3 ? 500.0 / 1113 - 7571.0 / 16695
         : j == 4 ? 125.0 / 192 - 393.0 / 640 : j == 5 ? -2187.0 / 6784 + 92097.0 / 339200
         : j == 6 ? 11.0 / 84 - 187.0 / 2100 : j == 7 ? -1.0 / 40 : 0.0;
}
// weight of k_j in the epilogue of DP45 stage S (next stage input, or the error at S = 7)
__host__ __device__ constexpr double dp_w(int S, int j) { return S == 7 ? dp_e(j) : dp_a(S + 1, j); }
__host__ __device__ constexpr double rk4_c(int s) { return s == 1 ? 0.0 : s == 4 ? 1.0 : 0.5; }

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

// block reduction of the DP45 error partials (256 threads = 4 waves): within
// each wave by lane exchanges, then the 4 wave results through LDS
__device__ __forceinline__ void reduce_partial(double sq, float mf, int nf, ErrPartial *out) {
    __shared__ double s_sq[4];
    __shared__ float s_mf[4];
    __shared__ int s_nf[4];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sq += __shfl_xor(sq, o, 64);
        mf = fmaxf(mf, __shfl_xor(mf, o, 64));
        nf |= __shfl_xor(nf, o, 64);
    }
    const int t = threadIdx.x, w = t >> 6;
    if ((t & 63) == 0) {
        s_sq[w] = sq;
        s_mf[w] = mf;
        s_nf[w] = nf;
    }
    __syncthreads();
    if (t == 0) {
        out->sumsq = (s_sq[0] + s_sq[1]) + (s_sq[2] + s_sq[3]);
        out->maxf = fmaxf(fmaxf(s_mf[0], s_mf[1]), fmaxf(s_mf[2], s_mf[3]));
        out->nonfinite = s_nf[0] | s_nf[1] | s_nf[2] | s_nf[3];
    }
}

// Does the neighbour at offset d (one axis, -1/0/+1) lie in the cell whose
// corner the node is at local index i (0/1) along that axis?
__host__ __device__ constexpr bool shares(int d, int i) { return d == 0 || (d == 1 && i == 0) || (d == -1 && i == 1); }

// q = floor(a / d) for 0 <= a < 2^20 from a float reciprocal rd ~ 1/d: the
// product is exact or one step low (never high: a / d is at least 1/a away
// from the next integer above it), so one correction suffices
__device__ __forceinline__ int small_div(int a, int d, float rd) {
    int q = (int)((float)a * rd);
    if (a - q * d >= d) ++q;
    return q;
}

// One thread per node (consecutive nodes along x, 256 per block).
//
// Neighbourhood.  With NIT > 0 the block first copies the m values it needs
// into LDS: for each z offset dz in {-1, 0, 1}, the nodes whose linear index
// lies within NX + 1 of (a node of the block + dz NX NY), a window of
// W = 256 + 2 NX + 2 nodes, stored as float4 {m_x, m_y, m_z, 0}; NIT items of
// the 3W per thread, read at clamped indices.  The neighbour at offsets
// (dx, dy, dz) of the block's thread t then sits at (dz + 1) W + t + NX + 1 +
// dy NX + dx (a single node layer, the film basis, keeps one window: its dz
// neighbours are the layer itself).  Every value is fetched from the caches
// once per block instead of by each of its 27 readers.  With NIT = 0 (rows too long for the window)
// every thread reads its 27 neighbours itself, at clamped indices.  A
// neighbour outside the mesh only enters through cells outside it, whose
// weight is 0, so whatever finite value its slot holds is harmless.
//
// Exchange is summed per neighbour d: m_d - m_n weighted by K^e at the
// axis-difference pattern of d times the sum of 2A over the cells holding
// both nodes (4 for a face neighbour, 2 for an edge, 1 for a corner), the
// cell-by-cell sum regrouped.  The Q1 mass matrix of a cuboid is a tensor
// product, M^e_ab = M^e(all axes differ) prod_k (2 if a_k = b_k else 1), so
// the anisotropy sum over the nodes b of cell q, sum_b M^e_ab (m_b . u_q), is
// u_q . S_q with S_q built by weighted pair sums along x, then y, then z;
// neighbouring cells share the partial sums.
//
// Loads are issued before any arithmetic, at clamped addresses with zero
// weights (a branch around a load makes each load its own round trip), the
// window loads first so that the LDS copy waits for them alone.  The stage
// is a template parameter, so every tableau coefficient is a compile-time
// constant.
#ifndef NM_NODE_WAVES
#define NM_NODE_WAVES 3
#endif
constexpr unsigned kNodeZGroup = 32;
// The node kernel's work for the 256-node range lb (the body shared by the
// single-mesh and the batched kernels).
// XT: the optional terms of this instantiation, a bit mask: 1 interfacial
// DMI, 2 bulk DMI, 4 cubic anisotropy
constexpr int kXtDmiI = 1, kXtDmiB = 2, kXtCubic = 4;
template <int MODE, int STAGE, int NIT, int XT>
__device__ __forceinline__ void node_body(const StencilParams &P, const StageArgs &S, unsigned lb) {
    const int tid = (int)threadIdx.x;
    const int n0 = (int)lb * 256;
    const int n = n0 + tid;
    const Ctrl *C = S.ctrl;
    const int nn = (int)P.nn;
    const int NX = P.NX, NY = P.NY, NZ = P.NZ, W = P.W;
    const int WS = NZ > 1 ? W : 0;   // LDS offset between the dz windows
    const float *in0 = S.in, *in1 = S.in + nn, *in2 = S.in + 2 * nn;

    // ---- LDS window of the stage input (issued first)
    __shared__ float4 sw[NIT > 0 ? NIT * 256 : 1];
    float wv[NIT > 0 ? NIT : 1][3];
    if constexpr (NIT > 0) {
        // window p starts at n0 - NX - 1 + (p - 1) NXY; NXY = 0 with one node
        // layer (the film basis), whose z neighbours are the layer itself:
        // the three windows coincide and only the first is kept (WS = 0)
        const int NXY = NZ > 1 ? NX * NY : 0;
        const int D = NXY - W;
        const int g0 = n0 - NX - 1 - NXY;          // = that start minus p W
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int j = tid + 256 * it;
            const int g = min(max(g0 + j + (j >= W ? D : 0) + (j >= 2 * W ? D : 0), 0), nn - 1);
            wv[it][0] = ldo(in0, 4u * (unsigned)g);
            wv[it][1] = ldo(in1, 4u * (unsigned)g);
            wv[it][2] = ldo(in2, 4u * (unsigned)g);
        }
    }

    // every thread computes (threads past the last node on the last one) so
    // that the whole block reaches the barrier; only real nodes store
    const bool valid = n < nn;
    const unsigned on = (unsigned)min(n, nn - 1) * 4u;   // byte offset of the node in one component
    const unsigned oc[3] = {on, on + 4u * (unsigned)nn, on + 8u * (unsigned)nn};
    constexpr int NK = MODE == kModeDP45 ? (STAGE > 1 ? STAGE - 1 : 1) : 1;
    float ms[3] = {0.f, 0.f, 0.f}, ac[3] = {0.f, 0.f, 0.f}, kk[NK][3];
    // ---- epilogue operands
    if (MODE == kModeRK4 || MODE == kModeDP45 || (MODE == kModeAdjFwd && STAGE < 4)) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ms[c] = ldo(S.mstate, oc[c]);
    }
    if (MODE == kModeRK4 && STAGE > 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ac[c] = ldo(S.acc, oc[c]);
    }
    float lo[3] = {0.f, 0.f, 0.f};
    if (MODE == kModeRK4 && STAGE == 4 && S.lo) {
#pragma unroll
        for (int c = 0; c < 3; ++c) lo[c] = ldo(S.lo, oc[c]);
    }
    if (MODE == kModeDP45) {
#pragma unroll
        for (int j = 0; j < NK; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                kk[j][c] = (j < STAGE - 1 && dp_w(STAGE, j + 1) != 0.0) ? ldo(S.k[j], oc[c]) : 0.f;
    }
    // ---- per-node coefficients
    const float im = ldo(P.inv_mass, on);
    float gp = 0.f, al = 0.f;
    if (MODE != kModeField) {
        gp = ldo(P.gp_n, on);
        al = ldo(P.alpha_n, on);
    }
    // ---- node coordinates from the block's first node (threads past the
    // end are moved onto the last plane)
    int x, y, z;
    {
        const int x0 = n0 % NX, r0 = n0 / NX;
        const int y0 = r0 % NY, z0 = r0 / NY;
        const int q1 = small_div(x0 + tid, NX, P.rNX);
        x = x0 + tid - q1 * NX;
        const int q2 = small_div(y0 + q1, NY, P.rNY);
        y = y0 + q1 - q2 * NY;
        z = min(z0 + q2, NZ - 1);
    }
    // ---- the 8 cells around the node, q = i1 + 2 i2 + 4 i3 for the cell
    // (x - i1, y - i2, z - i3), at clamped indices with weight cw = 0
    // outside the mesh
    float cw[8];
    unsigned co[8];
    float4 cp[8], cs[8];
    {
        const int N1 = P.N1, N2 = P.N2, N3 = P.N3;
        const unsigned ox[2] = {(unsigned)min(x, N1 - 1), (unsigned)max(x - 1, 0)};
        const unsigned oy[2] = {(unsigned)min(y, N2 - 1) * (unsigned)N1, (unsigned)max(y - 1, 0) * (unsigned)N1};
        const unsigned oz[2] = {(unsigned)min(z, N3 - 1) * (unsigned)(N1 * N2),
                                (unsigned)min(max(z - 1, 0), N3 - 1) * (unsigned)(N1 * N2)};
        const float fx[2] = {x < N1 ? 1.f : 0.f, x > 0 ? 1.f : 0.f};
        const float fy[2] = {y < N2 ? 1.f : 0.f, y > 0 ? 1.f : 0.f};
        const float fz[2] = {z < N3 ? 1.f : 0.f, z > 0 ? 1.f : 0.f};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i1 = q & 1, i2 = (q >> 1) & 1, i3 = q >> 2;
            co[q] = 16u * (oz[i3] + oy[i2] + ox[i1]);
            cw[q] = fx[i1] * fy[i2] * fz[i3];
            cp[q] = ldo(P.cellP, co[q]);
        }
    }
    // DMI constants weighted like the cells (0 outside the mesh)
    float dq[8];
    if constexpr ((XT & (kXtDmiI | kXtDmiB)) != 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) dq[q] = cw[q] * ldo(P.Dc, co[q] >> 2);
    }
    if (P.src) {
#pragma unroll
        for (int q = 0; q < 8; ++q) cs[q] = ldo(P.src, co[q]);
    } else {
#pragma unroll
        for (int q = 0; q < 8; ++q) cs[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // ---- the step clock: a finished controller turns the kernel into a
    // no-op; it is read after the loads above are issued, so its round trip
    // overlaps theirs
    double t, dt;
    {
        constexpr double cst = MODE == kModeDP45 ? dp_c(STAGE)
                             : (MODE == kModeRK4 || MODE == kModeAdjFwd) ? rk4_c(STAGE) : 0.0;
        if (C) {
            if (C->done) return;
            dt = C->dt;
            t = C->t + cst * dt;
        } else {
            dt = S.dt0;
            t = S.t0 + cst * dt;
        }
    }
    // ---- neighbourhood
    float v[NIT > 0 ? 1 : 27][3];
    int lrow[9];
    if constexpr (NIT > 0) {
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int j = tid + 256 * it;
            if (j < (NZ > 1 ? 3 : 1) * W) sw[j] = make_float4(wv[it][0], wv[it][1], wv[it][2], 0.f);
        }
        // row starts (dx = -1) of the 9 (dz, dy) neighbour rows in the window
#pragma unroll
        for (int k = 0; k < 9; ++k) lrow[k] = tid + NX + (k / 3) * WS + (k % 3 - 1) * NX;
        __syncthreads();
    } else {
        int cx[3], cy[3], cz[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            cx[d] = min(max(x + d - 1, 0), NX - 1);
            cy[d] = min(max(y + d - 1, 0), NY - 1) * NX;
            cz[d] = min(max(z + d - 1, 0), NZ - 1) * NX * NY;
        }
#pragma unroll
        for (int k = 0; k < 27; ++k) {
            const unsigned o = 4u * (unsigned)(cz[k / 9] + cy[(k / 3) % 3] + cx[k % 3]);
            v[k][0] = ldo(in0, o);
            v[k][1] = ldo(in1, o);
            v[k][2] = ldo(in2, o);
        }
    }
    // neighbour (dx, dy, dz) = (k % 3 - 1, (k / 3) % 3 - 1, k / 9 - 1)
    auto nb = [&](int k) -> float4 {
        if constexpr (NIT > 0)
            return sw[lrow[k / 3] + k % 3];
        else
            return make_float4(v[k][0], v[k][1], v[k][2], 0.f);
    };

    float r0 = 0.f, r1 = 0.f, r2 = 0.f, wd = 0.f;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        r0 += cw[q] * cs[q].x;
        r1 += cw[q] * cs[q].y;
        r2 += cw[q] * cs[q].z;
        wd += cw[q] * cs[q].w;
    }
    if (P.drive) {
        wd *= (float)sin(2.0 * 3.14159265358979323846 * P.dfreq * t + P.dphase);
        r0 += wd * P.damp[0];
        r1 += wd * P.damp[1];
        r2 += wd * P.damp[2];
    }
    const float4 mn = nb(13);
    const bool ex = P.terms & NM_T_EXCHANGE;
    const bool an = (P.terms & NM_T_ANIS) != 0;
    // cp = {2A carrying the sign of Ku, u = sqrt|Ku| e}
    float a2[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) a2[q] = cw[q] * fabsf(cp[q].x);
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    // anisotropy partial sums: S[q] = sum_b 2^(3 - #differing axes) m_b over cell q
    float3 Sq[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) Sq[q] = make_float3(0.f, 0.f, 0.f);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
        float4 vb[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) vb[k] = nb((dz + 1) * 9 + k);
        // exchange: edge and corner neighbours, then (K^e of a cube gives
        // them weight 0) the face neighbours unless the cells are cubes
        auto exch = [&](int dx, int dy) {
            float as = 0.f;
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (shares(dx, q & 1) && shares(dy, (q >> 1) & 1) && shares(dz, q >> 2)) as += a2[q];
            const int mask = (dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2);
            const float w = as * P.Kp[mask];
            const float4 b = vb[(dy + 1) * 3 + dx + 1];
            g0 += w * (b.x - mn.x);
            g1 += w * (b.y - mn.y);
            g2 += w * (b.z - mn.z);
        };
        if (ex) {
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx)
                    if ((dx != 0) + (dy != 0) + (dz != 0) >= 2) exch(dx, dy);
            if (P.faces) {
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx)
                        if ((dx != 0) + (dy != 0) + (dz != 0) == 1) exch(dx, dy);
            }
        }
        if (an) {
            // x pairs of the three rows: cell side i1 = 0 pairs x with x + 1, i1 = 1 with x - 1
            float3 tx[2][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int i1 = 0; i1 < 2; ++i1) {
                    const float4 c = vb[r * 3 + 1], o = vb[r * 3 + (i1 ? 0 : 2)];
                    tx[i1][r] = make_float3(2.f * c.x + o.x, 2.f * c.y + o.y, 2.f * c.z + o.z);
                }
#pragma unroll
            for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
                for (int i2 = 0; i2 < 2; ++i2) {
                    const float3 c = tx[i1][1], o = tx[i1][i2 ? 0 : 2];
                    const float3 ty = make_float3(2.f * c.x + o.x, 2.f * c.y + o.y, 2.f * c.z + o.z);
                    const int q0 = i1 + 2 * i2, q1 = q0 + 4;   // cells below (i3 = 0) / above (i3 = 1)
                    if (dz == -1) {
                        Sq[q1] = ty;
                    } else if (dz == 0) {
                        Sq[q1] = make_float3(Sq[q1].x + 2.f * ty.x, Sq[q1].y + 2.f * ty.y, Sq[q1].z + 2.f * ty.z);
                        Sq[q0] = make_float3(2.f * ty.x, 2.f * ty.y, 2.f * ty.z);
                    } else {
                        Sq[q0] = make_float3(Sq[q0].x + ty.x, Sq[q0].y + ty.y, Sq[q0].z + ty.z);
                    }
                }
        }
        if constexpr ((XT & (kXtDmiI | kXtDmiB)) != 0) {
            // A_k(a, b) = G_k(a, b) - G_k(b, a) = d_k times the 1D mass factors
            // of the other two axes (gx, gy, gz indexed by which of them
            // differ): the same in every cell holding both nodes, so per
            // neighbour d it is weighted by the sum of D over those cells.
            // Interfacial: g += (-A_x m_z, -A_y m_z, A_x m_x + A_y m_y);
            // bulk: g_j += eps_jkl A_k m_l
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    if (dx == 0 && dy == 0 && ((XT & kXtDmiI) || dz == 0)) continue;
                    float ds = 0.f;
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        if (shares(dx, q & 1) && shares(dy, (q >> 1) & 1) && shares(dz, q >> 2)) ds += dq[q];
                    const float wx = dx == 0 ? 0.f : ds * (float)dx * P.gx[(dy != 0) + 2 * (dz != 0)];
                    const float wy = dy == 0 ? 0.f : ds * (float)dy * P.gy[(dx != 0) + 2 * (dz != 0)];
                    const float4 b = vb[(dy + 1) * 3 + dx + 1];
                    if constexpr (XT & kXtDmiI) {
                        g0 -= wx * b.z;
                        g1 -= wy * b.z;
                        g2 += wx * b.x + wy * b.y;
                    } else {
                        const float wz = dz == 0 ? 0.f : ds * (float)dz * P.gz[(dx != 0) + 2 * (dy != 0)];
                        g0 += wy * b.z - wz * b.y;
                        g1 += wz * b.x - wx * b.z;
                        g2 += wx * b.y - wy * b.x;
                    }
                }
        }
    }
    if constexpr ((XT & kXtCubic) != 0) {
        // cubic anisotropy, quartic in m: Kc sum_g w phi_a(x_g) df/dm(m^h(x_g))
        // over the 2-point Gauss points x_g of each cell q holding the node,
        // a = (i1, i2, i3) the node's corner of q, m^h(x_g) interpolated from
        // the cell's 8 corners (node offsets b - a) axis by axis
        const float xi[2] = {P.gq[0], P.gq[1]};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i1 = q & 1, i2 = (q >> 1) & 1, i3 = q >> 2;
            const float4 k0 = ldo(P.cubP, 2u * co[q]), k1 = ldo(P.cubP, 2u * co[q] + 16u);
            const float kc = k0.x * cw[q] * P.gw;
            const float c1[3] = {k0.y, k0.z, k0.w}, c2[3] = {k1.x, k1.y, k1.z};
            const float c3[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                                 c1[0] * c2[1] - c1[1] * c2[0]};
            // corner values, then interpolation along x, y, z to the Gauss points
            float cv[8][3];
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const float4 t = nb(((b >> 2) - i3 + 1) * 9 + (((b >> 1) & 1) - i2 + 1) * 3 + ((b & 1) - i1 + 1));
                cv[b][0] = t.x;
                cv[b][1] = t.y;
                cv[b][2] = t.z;
            }
            float gv[8][3];
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const float wgt[3] = {xi[g & 1], xi[(g >> 1) & 1], xi[g >> 2]};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float yz[4];
#pragma unroll
                    for (int r = 0; r < 4; ++r) yz[r] = cv[2 * r][c] + wgt[0] * (cv[2 * r + 1][c] - cv[2 * r][c]);
                    const float z0 = yz[0] + wgt[1] * (yz[1] - yz[0]), z1 = yz[2] + wgt[1] * (yz[3] - yz[2]);
                    gv[g][c] = z0 + wgt[2] * (z1 - z0);
                }
            }
            float acc0 = 0.f, acc1 = 0.f, acc2 = 0.f;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const float a1 = gv[g][0] * c1[0] + gv[g][1] * c1[1] + gv[g][2] * c1[2];
                const float a2 = gv[g][0] * c2[0] + gv[g][1] * c2[1] + gv[g][2] * c2[2];
                const float a3 = gv[g][0] * c3[0] + gv[g][1] * c3[1] + gv[g][2] * c3[2];
                const float s1 = a1 * a1, s2 = a2 * a2, s3 = a3 * a3;
                // phi_a at x_g: psi_{a_k}(x_g,k) = x or 1 - x
                const float ph = (i1 ? xi[g & 1] : 1.f - xi[g & 1]) * (i2 ? xi[(g >> 1) & 1] : 1.f - xi[(g >> 1) & 1]) *
                                 (i3 ? xi[g >> 2] : 1.f - xi[g >> 2]);
                const float f1 = 2.f * a1 * (s2 + s3) * ph, f2 = 2.f * a2 * (s3 + s1) * ph, f3 = 2.f * a3 * (s1 + s2) * ph;
                acc0 += f1 * c1[0] + f2 * c2[0] + f3 * c3[0];
                acc1 += f1 * c1[1] + f2 * c2[1] + f3 * c3[1];
                acc2 += f1 * c1[2] + f2 * c2[2] + f3 * c3[2];
            }
            g0 += kc * acc0;
            g1 += kc * acc1;
            g2 += kc * acc2;
        }
    }
    if (an) {
        const float m7 = P.Mp[7];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            // -2 Ku e (sum M m . e) = -2 sign(Ku) u (sum M m . u)
            const float dot = cp[q].y * Sq[q].x + cp[q].z * Sq[q].y + cp[q].w * Sq[q].z;
            const float f2 = (signbit(cp[q].x) ? -2.f : 2.f) * m7 * cw[q] * dot;
            g0 -= f2 * cp[q].y;
            g1 -= f2 * cp[q].z;
            g2 -= f2 * cp[q].w;
        }
    }
    const float mv[3] = {mn.x, mn.y, mn.z};
    const float H[3] = {(r0 - g0) * im, (r1 - g1) * im, (r2 - g2) * im};
    float f[3] = {0.f, 0.f, 0.f};
    if (MODE != kModeField) llg_rhs(mv, H, gp, al, f);
    double sq = 0.0;
    float mf = 0.f;
    int nf = 0;
    if (valid) {
        if (MODE == kModeField) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sto(S.out, oc[c], H[c]);
        } else if (MODE == kModeAdjFwd) {
            // H(y_s) for the reverse sweep, y_{s+1} = m + c_{s+1} dt f_s
            const float cy = (float)(dt * (STAGE == 3 ? 1.0 : 0.5));
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sto(S.out, oc[c], H[c]);
                if (STAGE < 4) sto(S.y_next, oc[c], ms[c] + cy * f[c]);
            }
        } else if (MODE == kModeRhs) {
#pragma unroll
            for (int c = 0; c < 3; ++c) sto(S.out, oc[c], f[c]);
        } else if (MODE == kModeRK4) {
            const float cy = (float)(dt * (STAGE == 3 ? 1.0 : 0.5));
            const float c6 = (float)(dt / 6.0);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (STAGE == 4) {
                    const float inc = c6 * (ac[c] + f[c]);
                    if (S.lo) {
                        // two-sum of state and increment (plus the carried low
                        // part): the rounding error of the float32 update is
                        // kept, not lost, so it does not accumulate over steps
                        const float b = inc + lo[c];
                        const float sum = ms[c] + b, bv = sum - ms[c];
                        sto(S.mstate, oc[c], sum);
                        sto(S.lo, oc[c], (ms[c] - (sum - bv)) + (b - bv));
                    } else {
                        sto(S.mstate, oc[c], ms[c] + inc);
                    }
                } else {
                    sto(S.acc, oc[c], STAGE == 1 ? f[c] : ac[c] + 2.f * f[c]);
                    sto(S.y_next, oc[c], ms[c] + cy * f[c]);
                }
            }
        } else {  // DP45: store k_s, then y_{s+1} or (s = 7) the scaled error
            float fn2 = 0.f;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                sto(S.k[STAGE - 1], oc[c], f[c]);
                float acc = (float)(dt * dp_w(STAGE, STAGE)) * f[c];
#pragma unroll
                for (int j = 0; j < STAGE - 1; ++j)
                    if (dp_w(STAGE, j + 1) != 0.0) acc += (float)(dt * dp_w(STAGE, j + 1)) * kk[j][c];
                if (STAGE < 7) {
                    sto(S.y_next, oc[c], ms[c] + acc);
                } else {
                    const float yn = mv[c];
                    const double sct = C->atol + C->rtol * fmax(fabs((double)ms[c]), fabs((double)yn));
                    const double rr = (double)acc / sct;
                    if (im > 0.f) sq += rr * rr;
                    if (!isfinite(acc) || !isfinite(yn)) nf = 1;
                    fn2 += f[c] * f[c];
                }
            }
            if (STAGE == 7 && im > 0.f) mf = sqrtf(fn2);
        }
    }
    if (MODE == kModeDP45 && STAGE == 7) reduce_partial(sq, mf, nf, S.partials + lb);
}

// The node range of block b of nb (the mesh's node blocks): consecutive
// block numbers on one XCD walk groups of kNodeZGroup 256-node ranges (a few
// rows of one node layer) layer by layer: the next layer's blocks find two of
// their three window layers and one of their two cell layers in that XCD's
// L2, while each block still reads contiguous rows.  zcols: ranges per
// layer; ranges past zcols NZ keep their place.
__device__ __forceinline__ unsigned node_range(unsigned b, unsigned nb, const StencilParams &P) {
    unsigned lb = xcd_block(b, nb);
    if (kNodeZGroup > 0 && lb < P.zcols * (unsigned)P.NZ) {
        const unsigned gi = lb / (kNodeZGroup * (unsigned)P.NZ);
        const unsigned w = min(kNodeZGroup, P.zcols - gi * kNodeZGroup);
        const unsigned rem = lb - gi * kNodeZGroup * (unsigned)P.NZ;
        lb = (rem / w) * P.zcols + gi * kNodeZGroup + rem % w;
    }
    return lb;
}

template <int MODE, int STAGE, int NIT, int XT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NIT > 0 ? NM_NODE_WAVES : 2, NIT > 0 ? NM_NODE_WAVES : 2)))
k_node(StencilParams P, StageArgs S) {
    node_body<MODE, STAGE, NIT, XT>(P, S, node_range(blockIdx.x, gridDim.x, P));
}

dim3 stencil_grid(const nm_mesh *m) { return dim3((unsigned)((m->n_nodes + 255) / 256)); }

// ---------------------------------------------------------------- energies
__global__ void __launch_bounds__(256) k_energy_cells(StencilParams P, const float *__restrict__ m,
                                                      double t, double *__restrict__ part) {
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    float eex = 0.f, ean = 0.f, ez = 0.f, ed = 0.f, edm = 0.f;
    if (c < P.nc) {
        const int cx = (int)(c % P.N1);
        const long long r = c / P.N1;
        const int cy = (int)(r % P.N2);
        const int cz = (int)(r / P.N2);
        float v[8][3];
        for (int b = 0; b < 8; ++b) {
            // the node layer above the cell (the same layer under the film basis)
            const long long nb = ((long long)min(cz + (b >> 2), P.NZ - 1) * P.NY + (cy + ((b >> 1) & 1))) * P.NX +
                                 cx + (b & 1);
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
        if ((P.terms & NM_T_DMI) && P.Dc) {
            // G_k(a,b) = (b_k - 1/2) gk[...] (1D mass factors of the other axes);
            // interfacial: D sum_ab [G_x(a,b) (m_az m_bx - m_ax m_bz) + G_y(a,b) (m_az m_by - m_ay m_bz)],
            // bulk: D sum_ab eps_jkl m_aj G_k(a,b) m_bl
            float s = 0.f;
            for (int a = 0; a < 8; ++a)
                for (int b = 0; b < 8; ++b) {
                    const int d = a ^ b;
                    const float gxv = ((b & 1) ? 0.5f : -0.5f) * P.gx[((d >> 1) & 1) + 2 * ((d >> 2) & 1)];
                    const float gyv = (((b >> 1) & 1) ? 0.5f : -0.5f) * P.gy[(d & 1) + 2 * ((d >> 2) & 1)];
                    if (!P.dmi_bulk) {
                        s += gxv * (v[a][2] * v[b][0] - v[a][0] * v[b][2]) +
                             gyv * (v[a][2] * v[b][1] - v[a][1] * v[b][2]);
                    } else {
                        const float gzv = ((b >> 2) ? 0.5f : -0.5f) * P.gz[(d & 1) + 2 * ((d >> 1) & 1)];
                        s += gyv * (v[a][0] * v[b][2] - v[a][2] * v[b][0]) +
                             gzv * (v[a][1] * v[b][0] - v[a][0] * v[b][1]) +
                             gxv * (v[a][2] * v[b][1] - v[a][1] * v[b][2]);
                    }
                }
            edm = P.Dc[c] * s;
        }
        if ((P.terms & NM_T_CUBIC) && P.cubP) {
            // Kc sum_g w f(m^h(x_g)) over the 2-point Gauss points, added to
            // the anisotropy energy
            const float4 k0 = P.cubP[2 * c], k1 = P.cubP[2 * c + 1];
            const float c1[3] = {k0.y, k0.z, k0.w}, c2[3] = {k1.x, k1.y, k1.z};
            const float c3[3] = {c1[1] * c2[2] - c1[2] * c2[1], c1[2] * c2[0] - c1[0] * c2[2],
                                 c1[0] * c2[1] - c1[1] * c2[0]};
            float s = 0.f;
            for (int g = 0; g < 8; ++g) {
                float mg[3] = {0.f, 0.f, 0.f};
                for (int b = 0; b < 8; ++b) {
                    float ph = 1.f;
                    for (int k = 0; k < 3; ++k) {
                        const float x = P.gq[(g >> k) & 1];
                        ph *= ((b >> k) & 1) ? x : 1.f - x;
                    }
                    for (int q = 0; q < 3; ++q) mg[q] += ph * v[b][q];
                }
                const float a1 = mg[0] * c1[0] + mg[1] * c1[1] + mg[2] * c1[2];
                const float a2 = mg[0] * c2[0] + mg[1] * c2[1] + mg[2] * c2[2];
                const float a3 = mg[0] * c3[0] + mg[1] * c3[1] + mg[2] * c3[2];
                s += a1 * a1 * a2 * a2 + a2 * a2 * a3 * a3 + a3 * a3 * a1 * a1;
            }
            ean += k0.x * P.gw * s;
        }
    }
    __shared__ double s[5][256];
    const int t0 = threadIdx.x;
    s[0][t0] = eex;
    s[1][t0] = ed;
    s[2][t0] = ean;
    s[3][t0] = ez;
    s[4][t0] = edm;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t0 < w)
            for (int k = 0; k < 5; ++k) s[k][t0] += s[k][t0 + w];
        __syncthreads();
    }
    if (t0 < 5) part[(long long)t0 * gridDim.x + blockIdx.x] = s[t0][0];
}

__global__ void k_energy_final(const double *__restrict__ part, int nb, double *__restrict__ out) {
    __shared__ double s[256];
    for (int k = 0; k < 5; ++k) {
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
// One block of 1024 threads: each thread sums a fixed strided subset of the
// block partials (8 loads in flight per round), then lane exchanges and LDS
// combine the 16 waves; the order is fixed, so the result is reproducible.
__device__ __forceinline__ void dp45_control_body(Ctrl *C, const ErrPartial *__restrict__ part, int np) {
    __shared__ double s_sq[16];
    __shared__ float s_mf[16];
    __shared__ int s_nf[16];
    const int t = threadIdx.x;
    double sq = 0.0;
    float mf = 0.f;
    int nf = 0;
    for (int i0 = 0; i0 < np; i0 += 8 * 1024) {
        ErrPartial q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * 1024 + t;
            q[u] = part[min(i, np - 1)];
            if (i >= np) q[u] = ErrPartial{0.0, 0.f, 0};
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            sq += q[u].sumsq;
            mf = fmaxf(mf, q[u].maxf);
            nf |= q[u].nonfinite;
        }
    }
    if (C->done) {
        if (t == 0) C->accept = 0;
        return;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        sq += __shfl_xor(sq, o, 64);
        mf = fmaxf(mf, __shfl_xor(mf, o, 64));
        nf |= __shfl_xor(nf, o, 64);
    }
    if ((t & 63) == 0) {
        s_sq[t >> 6] = sq;
        s_mf[t >> 6] = mf;
        s_nf[t >> 6] = nf;
    }
    __syncthreads();
    if (t != 0) return;
    double tsq = 0.0;
    float tmf = 0.f;
    int tnf = 0;
    for (int w = 0; w < 16; ++w) {
        tsq += s_sq[w];
        tmf = fmaxf(tmf, s_mf[w]);
        tnf |= s_nf[w];
    }
    s_sq[0] = tsq;
    s_mf[0] = tmf;
    s_nf[0] = tnf;
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

__global__ void __launch_bounds__(1024) k_dp45_control(Ctrl *C, const ErrPartial *__restrict__ part, int np) {
    dp45_control_body(C, part, np);
}

__device__ __forceinline__ void dp45_finish_body(const Ctrl *__restrict__ C, float *__restrict__ mstate,
                                                 const float *__restrict__ y7, float *__restrict__ k1,
                                                 const float *__restrict__ k7, float *__restrict__ y2,
                                                 long long n3, double a21, long long i) {
    if (i >= n3) return;
    const bool acc = C->accept;
    const bool done = C->done;
    if (!acc && done) return;
    // accepted: the 5th-order solution and k7 become the state and k1
    // (first same as last); rejected: both stay
    float mv, kv;
    if (acc) {
        mv = y7[i];
        kv = k7[i];
        mstate[i] = mv;
        k1[i] = kv;
    } else {
        mv = mstate[i];
        kv = k1[i];
    }
    if (!done) y2[i] = mv + (float)(C->dt * a21) * kv;
}

__global__ void k_dp45_finish(const Ctrl *__restrict__ C, float *__restrict__ mstate,
                              const float *__restrict__ y7, float *__restrict__ k1,
                              const float *__restrict__ k7, float *__restrict__ y2, long long n3,
                              double a21) {
    dp45_finish_body(C, mstate, y7, k1, k7, y2, n3, a21, (long long)blockIdx.x * 256 + threadIdx.x);
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
    P.cellP = m->cellP;
    // source of the node kernel: the demag pass writes mu0 Ms V/8 (H_d [+ static
    // H_ext]) into hd; without demag the static Zeeman part is read directly
    P.src = (terms & NM_T_DEMAG) ? reinterpret_cast<const float4 *>(m->hd)
                                 : ((terms & NM_T_ZEEMAN) ? m->wstat : nullptr);
    P.drive = ((terms & NM_T_ZEEMAN) && m->has_drive) ? 1 : 0;
    P.W = 256 + 2 * m->NX + 2;
    P.faces = (m->Kp[1] != 0.f || m->Kp[2] != 0.f || m->Kp[4] != 0.f) ? 1 : 0;
    P.zcols = m->NZ > 1 ? stencil_grid(m).x / (unsigned)m->NZ : 0u;
    P.Dc = ((terms & NM_T_DMI) && m->has_dmi) ? m->Dc : nullptr;
    P.dmi_bulk = m->dmi_bulk ? 1 : 0;
    for (int i = 0; i < 4; ++i) {
        P.gx[i] = m->gx[i];
        P.gy[i] = m->gy[i];
        // a single node layer (the film basis) has no derivative along z
        P.gz[i] = m->NZ > 1 ? m->gz[i] : 0.f;
    }
    P.cubP = ((terms & NM_T_CUBIC) && m->has_cubic) ? m->cubP : nullptr;
    P.gq[0] = m->gq[0];
    P.gq[1] = m->gq[1];
    P.gw = m->gw;
    P.rNX = 1.f / (float)m->NX;
    P.rNY = 1.f / (float)m->NY;
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

// window items per thread: the smallest of 5, 7, 10, 13 covering the 3 W of
// the dz windows (one W with a single node layer); longer rows (NX > 425,
// or NX > 1535 with one layer) read their neighbours directly
int window_items(int NX, int NZ) {
    const int need = ((NZ > 1 ? 3 : 1) * (256 + 2 * NX + 2) + 255) / 256;
    return need <= 5 ? 5 : need <= 7 ? 7 : need <= 10 ? 10 : need <= 13 ? 13 : 0;
}

// The optional terms are separate instantiations, so meshes without them
// keep the register budget of the others.  Interfacial DMI takes the LDS
// window up to 10 items (the 13-item window would spill at 3 waves per
// SIMD); bulk DMI and cubic anisotropy read their neighbours directly.
template <int MODE, int STAGE, int XT>
static void launch_node_t(nm_mesh *m, dim3 grid, const StencilParams &P, const StageArgs &S) {
    const int nit = (XT & ~kXtDmiI) ? 0 : window_items(m->NX, m->NZ);
    switch (nit) {
        case 5:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                NM_LAUNCH(m, NM_PROF_STENCIL, (k_node<MODE, STAGE, 5, XT>), grid, dim3(256), 0, P, S);
                break;
            }
            [[fallthrough]];
        case 7:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                NM_LAUNCH(m, NM_PROF_STENCIL, (k_node<MODE, STAGE, 7, XT>), grid, dim3(256), 0, P, S);
                break;
            }
            [[fallthrough]];
        case 10:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                NM_LAUNCH(m, NM_PROF_STENCIL, (k_node<MODE, STAGE, 10, XT>), grid, dim3(256), 0, P, S);
                break;
            }
            [[fallthrough]];
        case 13:
            if constexpr (XT == 0) {
                NM_LAUNCH(m, NM_PROF_STENCIL, (k_node<MODE, STAGE, 13, 0>), grid, dim3(256), 0, P, S);
                break;
            }
            [[fallthrough]];
        default: NM_LAUNCH(m, NM_PROF_STENCIL, (k_node<MODE, STAGE, 0, XT>), grid, dim3(256), 0, P, S); break;
    }
}

// the node kernel's term instantiation for parameters P (kXt* bits)
static int params_xt(const StencilParams &P) {
    return (P.Dc ? (P.dmi_bulk ? kXtDmiB : kXtDmiI) : 0) | (P.cubP ? kXtCubic : 0);
}

int node_xt(const nm_mesh *m, unsigned terms) { return params_xt(make_params(m, terms)); }

template <int MODE, int STAGE>
static void launch_node(nm_mesh *m, dim3 grid, const StencilParams &P, const StageArgs &S) {
    switch (params_xt(P)) {
        case 0: launch_node_t<MODE, STAGE, 0>(m, grid, P, S); break;
        case kXtDmiI: launch_node_t<MODE, STAGE, kXtDmiI>(m, grid, P, S); break;
        case kXtDmiB: launch_node_t<MODE, STAGE, kXtDmiB>(m, grid, P, S); break;
        case kXtCubic: launch_node_t<MODE, STAGE, kXtCubic>(m, grid, P, S); break;
        case kXtCubic | kXtDmiI: launch_node_t<MODE, STAGE, kXtCubic | kXtDmiI>(m, grid, P, S); break;
        default: launch_node_t<MODE, STAGE, kXtCubic | kXtDmiB>(m, grid, P, S); break;
    }
}

hipError_t launch_stencil(nm_mesh *m, unsigned terms, const StageSpec &sp) {
    StencilParams P = make_params(m, terms);
    StageArgs S{};
    S.in = sp.in;
    S.out = sp.out;
    S.y_next = sp.y_next;
    S.mstate = sp.mstate;
    S.acc = m->acc;
    S.lo = sp.lo;
    S.t0 = sp.t0;
    S.dt0 = sp.dt0;
    S.ctrl = sp.use_ctrl ? m->ctrl : nullptr;
    S.partials = m->partials;
    for (int j = 0; j < 7; ++j) S.k[j] = m->k[j];
    const dim3 g = stencil_grid(m);
    if (sp.mode == kModeField) {
        launch_node<kModeField, 0>(m, g, P, S);
    } else if (sp.mode == kModeRhs) {
        launch_node<kModeRhs, 0>(m, g, P, S);
    } else if (sp.mode == kModeAdjFwd) {
        switch (sp.stage) {
            case 1: launch_node<kModeAdjFwd, 1>(m, g, P, S); break;
            case 2: launch_node<kModeAdjFwd, 2>(m, g, P, S); break;
            case 3: launch_node<kModeAdjFwd, 3>(m, g, P, S); break;
            case 4: launch_node<kModeAdjFwd, 4>(m, g, P, S); break;
            default: return hipErrorInvalidValue;
        }
    } else if (sp.mode == kModeRK4) {
        switch (sp.stage) {
            case 1: launch_node<kModeRK4, 1>(m, g, P, S); break;
            case 2: launch_node<kModeRK4, 2>(m, g, P, S); break;
            case 3: launch_node<kModeRK4, 3>(m, g, P, S); break;
            case 4: launch_node<kModeRK4, 4>(m, g, P, S); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (sp.stage) {
            case 1: launch_node<kModeDP45, 1>(m, g, P, S); break;
            case 2: launch_node<kModeDP45, 2>(m, g, P, S); break;
            case 3: launch_node<kModeDP45, 3>(m, g, P, S); break;
            case 4: launch_node<kModeDP45, 4>(m, g, P, S); break;
            case 5: launch_node<kModeDP45, 5>(m, g, P, S); break;
            case 6: launch_node<kModeDP45, 6>(m, g, P, S); break;
            case 7: launch_node<kModeDP45, 7>(m, g, P, S); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_energy(nm_mesh *m, const float *mag, unsigned terms, double t, double e[6]) {
    StencilParams P = make_params(m, terms);
    const unsigned grid = (unsigned)((m->n_cells + 255) / 256);
    if ((int)grid > m->n_eblocks) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_energy_cells, dim3(grid), dim3(256), 0, m->stream, P, mag, t, m->ered);
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, m->stream, m->ered, (int)grid,
                       m->ered + 5LL * m->n_eblocks);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    double host[5];
    err = hipMemcpyAsync(host, m->ered + 5LL * m->n_eblocks, sizeof(host), hipMemcpyDeviceToHost,
                         m->stream);
    if (err == hipSuccess) err = hipStreamSynchronize(m->stream);
    if (err != hipSuccess) return err;
    for (int k = 0; k < 4; ++k) e[k] = host[k];
    e[5] = host[4];
    e[4] = host[0] + host[1] + host[2] + host[3] + host[4];
    return hipSuccess;
}

hipError_t launch_dp45_control(nm_mesh *m) {
    const int np = (int)stencil_grid(m).x;
    NM_LAUNCH(m, NM_PROF_CONTROL, k_dp45_control, dim3(1), dim3(1024), 0, m->ctrl, m->partials, np);
    return hipGetLastError();
}

hipError_t launch_dp45_finish(nm_mesh *m, float *mstate) {
    const double a21 = dp_a(2, 1);
    const long long n3 = 3 * m->n_nodes;
    NM_LAUNCH(m, NM_PROF_CONTROL, k_dp45_finish, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0,
              m->ctrl, mstate, m->y[1], m->k[0], m->k[6], m->y[0], n3, a21);
    return hipGetLastError();
}

// packed node-kernel data from the raw cell copies (mesh creation, new field map)
__global__ void k_cell_pack(const float *__restrict__ A2, const float *__restrict__ Ku,
                            const float *__restrict__ easy, const float *__restrict__ wc,
                            const float *__restrict__ hcell, const float *__restrict__ dmask,
                            float hu0, float hu1, float hu2, float4 *__restrict__ cellP,
                            float4 *__restrict__ wstat, long long nc) {
    const long long c = (long long)blockIdx.x * 256 + threadIdx.x;
    if (c >= nc) return;
    float u0 = 0.f, u1 = 0.f, u2 = 0.f, k = 0.f;
    if (Ku) {
        k = Ku[c];
        const float r = sqrtf(fabsf(k));
        u0 = r * easy[c];
        u1 = r * easy[nc + c];
        u2 = r * easy[2 * nc + c];
    }
    const float w = wc[c];
    // 2A >= 0, so its sign bit is free to carry the sign of Ku (easy axis or
    // easy plane): Ku e (m . e) = sign(Ku) u (m . u) with u = sqrt|Ku| e
    cellP[c] = make_float4(copysignf(A2[c], k), u0, u1, u2);
    float h0 = hu0, h1 = hu1, h2 = hu2;
    if (hcell) {
        h0 += hcell[c];
        h1 += hcell[nc + c];
        h2 += hcell[2 * nc + c];
    }
    wstat[c] = make_float4(w * h0, w * h1, w * h2, dmask ? w * dmask[c] : 0.f);
}

hipError_t launch_cell_pack(nm_mesh *m) {
    const long long nc = m->n_cells;
    hipLaunchKernelGGL(k_cell_pack, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, m->stream, m->A2,
                       m->has_anis ? m->Ku : nullptr, m->easy, m->wc, m->has_hcell ? m->h_cell : nullptr,
                       m->has_drive ? m->drive_mask : nullptr, m->h_uniform[0], m->h_uniform[1],
                       m->h_uniform[2], m->cellP, m->wstat, nc);
    return hipGetLastError();
}

hipError_t launch_rk4_advance(nm_mesh *m) {
    NM_LAUNCH(m, NM_PROF_CONTROL, k_rk4_advance, dim3(1), dim3(1), 0, m->ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------ batched launches
// One launch covers every slot of a batch group (grid z = slot).  Each block
// runs exactly the code of the single-mesh kernel on its slot's buffers, so a
// solve's result does not depend on the other solves of its group.  The
// first np blocks of a slot (its own node blocks) take node ranges as the
// single-mesh launch does; the dispatcher deals them over the XCDs in the
// same rotation, shifted by the slot's place in the grid, which keeps each
// XCD on one contiguous range.
template <int STAGE, int NIT, int XT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(NIT > 0 ? NM_NODE_WAVES : 2, NIT > 0 ? NM_NODE_WAVES : 2)))
k_node_b(const BatchSlot *__restrict__ slots) {
    const BatchSlot &d = slots[blockIdx.z];
    if (!d.active || blockIdx.x >= (unsigned)d.np) return;
    node_body<kModeDP45, STAGE, NIT, XT>(d.P, d.S[STAGE], node_range(blockIdx.x, (unsigned)d.np, d.P));
}

__global__ void __launch_bounds__(1024) k_dp45_control_b(const BatchSlot *__restrict__ slots) {
    const BatchSlot &d = slots[blockIdx.x];
    if (!d.active) return;
    dp45_control_body(d.ctrl, d.partials, d.np);
}

__global__ void k_dp45_finish_b(const BatchSlot *__restrict__ slots, double a21) {
    const BatchSlot &d = slots[blockIdx.z];
    if (!d.active) return;
    dp45_finish_body(d.ctrl, d.mstate, d.y1, d.k1, d.k7, d.y0, d.n3, a21,
                     (long long)blockIdx.x * 256 + threadIdx.x);
}

// descriptor of one solve: mesh m with its state mstate, the buffers as the
// DP45 stepping of nm_llg_step uses them; ctrl: the controller the batched
// kernels update
void batch_slot_fill(const nm_mesh *m, unsigned terms, Ctrl *ctrl, float *mstate, BatchSlot *out) {
    BatchSlot d{};
    d.active = 1;
    d.N1 = m->N1;
    d.N2 = m->N2;
    d.N3 = m->N3;
    d.NZ = m->NZ;
    d.P2 = m->P2;
    d.K1 = m->K1;
    d.KP = m->KP;
    d.P2h = m->P2h;
    d.P3h = m->P3h;
    d.src_mode = (terms & NM_T_ZEEMAN) ? 2 : 1;
    d.Ms = m->Ms;
    d.spec = m->spec;
    d.tensor = m->tensor;
    d.hd = m->hd;
    d.wc = m->wc;
    d.wstat = m->wstat;
    d.ctrl = ctrl;
    d.partials = m->partials;
    d.np = (int)stencil_grid(m).x;
    d.y0 = m->y[0];
    d.y1 = m->y[1];
    d.k1 = m->k[0];
    d.k7 = m->k[6];
    d.n3 = 3 * m->n_nodes;
    d.P = make_params(m, terms);
    d.mstate = mstate;
    for (int st = 2; st <= 7; ++st) {
        d.stage_in[st] = m->y[st % 2];
        StageArgs &S = d.S[st];
        S.in = m->y[st % 2];
        S.out = nullptr;
        S.y_next = st < 7 ? m->y[(st + 1) % 2] : nullptr;
        S.mstate = mstate;
        S.acc = m->acc;
        S.ctrl = ctrl;
        S.partials = m->partials;
        for (int j = 0; j < 7; ++j) S.k[j] = m->k[j];
        S.t0 = S.dt0 = 0.0;
    }
    *out = d;
}

// the window sizes each term instantiation takes, as for a single mesh
// (launch_node_t): interfacial DMI up to 10 items, the other extra terms none
template <int STAGE, int XT>
static void launch_node_bx(const BatchClass &bc, const BatchSlot *slots, int cap, hipStream_t st) {
    const dim3 g(bc.node_blocks, 1, (unsigned)cap);
    const int nit = (XT & ~kXtDmiI) ? 0 : bc.nit;
    switch (nit) {
        case 5:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                hipLaunchKernelGGL((k_node_b<STAGE, 5, XT>), g, dim3(256), 0, st, slots);
                break;
            }
            [[fallthrough]];
        case 7:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                hipLaunchKernelGGL((k_node_b<STAGE, 7, XT>), g, dim3(256), 0, st, slots);
                break;
            }
            [[fallthrough]];
        case 10:
            if constexpr ((XT & ~kXtDmiI) == 0) {
                hipLaunchKernelGGL((k_node_b<STAGE, 10, XT>), g, dim3(256), 0, st, slots);
                break;
            }
            [[fallthrough]];
        case 13:
            if constexpr (XT == 0) {
                hipLaunchKernelGGL((k_node_b<STAGE, 13, 0>), g, dim3(256), 0, st, slots);
                break;
            }
            [[fallthrough]];
        default: hipLaunchKernelGGL((k_node_b<STAGE, 0, XT>), g, dim3(256), 0, st, slots); break;
    }
}

template <int STAGE>
static void launch_node_b(const BatchClass &bc, const BatchSlot *slots, int cap, hipStream_t st) {
    switch (bc.xt) {
        case 0: launch_node_bx<STAGE, 0>(bc, slots, cap, st); break;
        case kXtDmiI: launch_node_bx<STAGE, kXtDmiI>(bc, slots, cap, st); break;
        case kXtDmiB: launch_node_bx<STAGE, kXtDmiB>(bc, slots, cap, st); break;
        case kXtCubic: launch_node_bx<STAGE, kXtCubic>(bc, slots, cap, st); break;
        case kXtCubic | kXtDmiI: launch_node_bx<STAGE, kXtCubic | kXtDmiI>(bc, slots, cap, st); break;
        default: launch_node_bx<STAGE, kXtCubic | kXtDmiB>(bc, slots, cap, st); break;
    }
}

hipError_t launch_batch_node(const BatchClass &bc, const BatchSlot *slots, int cap, int stage, hipStream_t st) {
    switch (stage) {
        case 2: launch_node_b<2>(bc, slots, cap, st); break;
        case 3: launch_node_b<3>(bc, slots, cap, st); break;
        case 4: launch_node_b<4>(bc, slots, cap, st); break;
        case 5: launch_node_b<5>(bc, slots, cap, st); break;
        case 6: launch_node_b<6>(bc, slots, cap, st); break;
        case 7: launch_node_b<7>(bc, slots, cap, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_control(const BatchSlot *slots, int cap, hipStream_t st) {
    hipLaunchKernelGGL(k_dp45_control_b, dim3((unsigned)cap), dim3(1024), 0, st, slots);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchClass &bc, const BatchSlot *slots, int cap, hipStream_t st) {
    const unsigned blocks = (unsigned)((3ull * bc.node_blocks * 256 + 255) / 256);
    hipLaunchKernelGGL(k_dp45_finish_b, dim3(blocks, 1, (unsigned)cap), dim3(256), 0, st, slots, dp_a(2, 1));
    return hipGetLastError();
}

}  // namespace nm
