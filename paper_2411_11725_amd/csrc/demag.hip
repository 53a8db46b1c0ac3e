// Demagnetisation field by zero-padded FFT convolution (Sec. 3.2), gfx950.
//
// Pipeline for a nodal magnetisation m (float32, SoA, x fastest):
//   x pass   nodal -> cell average M_c = Ms_c (1/8) sum of the 8 corners (the
//            exact cell mean of the trilinear m^h), real-to-complex FFT along
//            x (length P1 through a complex FFT of length P1/2), only the N2 N3
//            non-zero rows;
//   y pass   complex FFT along y of the N3 non-zero z planes (3D), rows >= N2
//            read as zeros;
//   z conv   FFT along z, H^ = -N^ M^ with the real symmetric k-space tensor,
//            inverse FFT along z, keeping the N3 planes (3D); for single-layer
//            films (N3 = 1) the same fusion happens along y instead;
//   y pass   inverse along y, keeping the N2 rows (3D);
//   x pass   complex-to-real along x, keeping the N1 cells -> cell field H_c.
// The spectrum lives in one workspace spec[3][N3][P2][KP] holding K1 = P1/2 + 1
// x frequencies per row, the row pitch KP rounded up to 16 complex (128 B) so
// that column tiles start on cache-line boundaries:
// every pass reads and writes whole column tiles in place, so no transposes
// are needed and loads / stores of a tile are contiguous along x.
// The tensor carries the 1/(P1 P2 P3) normalisation of the inverse transform.
// Transforms: the x passes sweep radix-8/4/2 Stockham passes through LDS
// (fft_engine.h); the y passes and the z convolution hold their pencils in
// registers and trade values once through LDS (fft2 in fft_reg.h), the z
// convolution applying the tensor in registers between its two transforms
// (P3 >= 512 falls back to the LDS sweep, as does the film convolution).
#include <map>
#include <mutex>
#include <tuple>

#include "fft_engine.h"
#include "fft_reg.h"

namespace nm {

__host__ __device__ constexpr int x_rows_per_block(int L) { return L >= 512 ? 1 : 512 / L; }

// Loads outside the live region are made at clamped addresses (always inside
// data written by the previous pass, hence finite) and zeroed by a 0/1 factor.
// A select or branch would let the compiler turn each load into a guarded one
// that waits for its own memory round trip; the factor keeps all loads of a
// thread in flight together.
__device__ __forceinline__ float2 keep(float2 v, bool ok) {
    const float f = ok ? 1.f : 0.f;
    return make_float2(v.x * f, v.y * f);
}

// ---------------------------------------------------------------- x forward
// block (by, z): the RB cell rows y0 <= y < y0 + RB of plane z.  A cell's
// value is Ms / 8 times the sum of its 8 corners: the block first sums the
// node pairs (z, z + 1) of its RB + 1 node rows into LDS (each node value is
// read once per block), then each cell adds four of those pair sums.
template <int L>
__device__ __forceinline__ void xfwd_body(const float *__restrict__ mag, const float *__restrict__ Ms,
                                          float2 *__restrict__ spec, const float2 *__restrict__ tw, int N1,
                                          int N2, int N3, int NZ, int P2, int KP, const Ctrl *__restrict__ ctrl,
                                          int bx, int by) {
    constexpr int RB = x_rows_per_block(L);
    constexpr int NP = 3 * RB;
    constexpr int NR = RB + 1, RL = L + 1;      // node rows; node slots per row (N1 + 1 <= L + 1)
    constexpr int NZI = 3 * NR * RL;            // pair sums: component, node row, node x
    constexpr int NA = (NZI + 255) / 256;
    __shared__ float2 s[NP * L];
    __shared__ float zs[NZI];
    __shared__ float2 tl[L + 1];   // exp(-2 pi i k / P1), k <= L
    const int tid = threadIdx.x;
    const int y0 = bx * RB, z = by;
    const int nrows = min(RB, N2 - y0);
    const int NX = N1 + 1, NY = N2 + 1;
    const unsigned nn = (unsigned)NX * NY * NZ;
    // node layer z + 1 of the cell layer z; the same layer under the film
    // basis (one node layer), which sums it twice: the mean of 4 corners
    const unsigned plane = NZ > 1 ? (unsigned)NX * NY : 0u;
    // node pair sums m(x, y, z) + m(x, y, z + 1), at clamped nodes (slots
    // past the row end and rows past the plane are never used unzeroed)
    float za[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        const int it = min(tid + 256 * a, NZI - 1);
        const int c = it / (NR * RL), rem = it - c * (NR * RL);
        const int jr = rem / RL, xn = rem - jr * RL;
        const unsigned o = 4u * (c * nn + ((unsigned)z * NY + (unsigned)min(y0 + jr, NY - 1)) * NX +
                                 (unsigned)min(xn, NX - 1));
        za[a] = ldo(mag, o) + ldo(mag, o + 4u * plane);
    }
    // Only the first L / 2 complex elements of a row hold cells (N1 <= P1 / 2);
    // the upper half is zero padding.  One thread per (row, element) of the
    // data half: RB L / 2 = 256.
    static_assert(RB * L / 2 == 256, "one data element per thread");
    const int rb = tid / (L / 2), n = tid - (tid / (L / 2)) * (L / 2);
    const bool rok = rb < nrows;
    const int y = y0 + min(rb, nrows - 1);
    float ms[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) ms[hh] = 0.125f * Ms[((long long)z * N2 + y) * N1 + min(2 * n + hh, N1 - 1)];
    // a finished controller turns the kernel into a no-op; the flag is read
    // after the data loads are issued, so its round trip overlaps theirs
    if (ctrl && ctrl->done) return;
#pragma unroll
    for (int a = 0; a < NA; ++a)
        if (tid + 256 * a < NZI) zs[tid + 256 * a] = za[a];
    __syncthreads();
    {
        float2 v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float *r0 = zs + (c * NR + rb) * RL + 2 * n, *r1 = r0 + RL;
            // cells 2n (nodes 2n, 2n + 1) and 2n + 1 (nodes 2n + 1, 2n + 2)
            const float p0 = r0[0] + r1[0], p1 = r0[1] + r1[1], p2 = r0[2] + r1[2];
            v[c].x = (rok && 2 * n < N1 ? 1.f : 0.f) * (ms[0] * (p0 + p1));
            v[c].y = (rok && 2 * n + 1 < N1 ? 1.f : 0.f) * (ms[1] * (p1 + p2));
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            s[(c * RB + rb) * L + n] = v[c];
            s[(c * RB + rb) * L + n + L / 2] = make_float2(0.f, 0.f);
        }
    }
    load_twiddles<2 * L, 256>(tl, tw, tid);
    __syncthreads();
    lds_fft<L, -1, NP, 256, false, 2 * L>(s, tl, tid);
    // untangle the half-length transform: X_k = E_k + W^k O_k, W = exp(-2 pi i / P1)
    for (int it = tid; it < RB * (L + 1); it += 256) {
        const int rb = it / (L + 1), k = it - (it / (L + 1)) * (L + 1);
        if (rb >= nrows) continue;
        const int y = y0 + rb;
        const float2 w = twiddle<-1>(tl, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 zk = s[(c * RB + rb) * L + (k & (L - 1))];
            const float2 zc = cconj(s[(c * RB + rb) * L + ((L - k) & (L - 1))]);
            const float2 e = cscale(cadd(zk, zc), 0.5f);
            const float2 d = cscale(csub(zk, zc), 0.5f);
            const float2 o = make_float2(d.y, -d.x);  // -i d
            sto(spec + (long long)c * N3 * P2 * KP, 8u * (((unsigned)z * (unsigned)P2 + (unsigned)y) * (unsigned)KP + (unsigned)k),
                cadd(e, cmul(w, o)));
        }
    }
}

// Block (row group, plane) of the x forward pass.  A block's last node row
// is the next block's first; with one cell row per block (L >= 512) that is
// half of what it reads, so the blocks go to the XCDs in contiguous ranges
// and the shared row comes from the XCD's L2 (the dispatcher hands
// consecutive blocks to different XCDs).  With several rows per block the
// dispatch order stays: plane-ordered ranges measured no faster there.
template <int L>
__device__ __forceinline__ void xfwd_block(int &bx, int &by) {
    if constexpr (x_rows_per_block(L) == 1) {
        const unsigned nx = gridDim.x, l = xcd_block(blockIdx.x + nx * blockIdx.y, nx * gridDim.y);
        bx = (int)(l % nx);
        by = (int)(l / nx);
    } else {
        bx = (int)blockIdx.x;
        by = (int)blockIdx.y;
    }
}

template <int L>
__global__ void __launch_bounds__(256)
k_xfwd(const float *__restrict__ mag, const float *__restrict__ Ms, float2 *__restrict__ spec,
       const float2 *__restrict__ tw, int N1, int N2, int N3, int NZ, int P2, int KP,
       const Ctrl *__restrict__ ctrl) {
    int bx, by;
    xfwd_block<L>(bx, by);
    xfwd_body<L>(mag, Ms, spec, tw, N1, N2, N3, NZ, P2, KP, ctrl, bx, by);
}

// ---------------------------------------------------------------- x inverse
template <int L>
__device__ __forceinline__ void xinv_body(const float2 *__restrict__ spec, float *__restrict__ hd,
                                          const float2 *__restrict__ tw, int N1, int N2, int N3, int P2, int KP,
                                          const float *__restrict__ wc, const float4 *__restrict__ wstat,
                                          int src_mode, const Ctrl *__restrict__ ctrl, int bx) {
    constexpr int RB = x_rows_per_block(L);
    constexpr int NP = 3 * RB;
    __shared__ float2 s[NP * L];
    __shared__ float2 tl[L + 1];   // exp(-2 pi i k / P1), k <= L
    const int tid = threadIdx.x;
    const int rows = N2 * N3;
    const int row0 = bx * RB;
    const long long nc = (long long)N1 * N2 * N3;
    static_assert((RB * L) % 256 == 0, "whole iterations");
    constexpr int NI = RB * L / 256;
    // input items (row rb, frequency k): NI per thread
    float2 xk[NI][3], xc[NI][3];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int it = tid + i * 256;
        const int rb = it / L, k = it - (it / L) * L;
        const int row = row0 + rb;
        const bool rok = row < rows;   // rows past the end: clamped read, zeroed
        const int rc = min(row, rows - 1);
        const int y = rc % N2, z = rc / N2;
        // 32-bit byte offset of the row within one component
        const unsigned ro = 8u * (((unsigned)z * (unsigned)P2 + (unsigned)y) * (unsigned)KP);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 *cb = spec + (long long)c * N3 * P2 * KP;
            xk[i][c] = keep(ldo(cb, ro + 8u * (unsigned)k), rok);
            xc[i][c] = keep(cconj(ldo(cb, ro + 8u * (unsigned)(L - k))), rok);
        }
    }
    // output items (row, cell x): only the first L / 2 complex elements of a
    // row are cells (N1 <= P1 / 2, element n holds cells 2n and 2n + 1), so
    // a block has RB L cells, two per thread, consecutive cells on
    // consecutive lanes; their weights and static fields are fetched now, at
    // clamped cells
    static_assert(RB * L == 512, "two output cells per thread");
    long long oi[2];
    int ol[2];
    bool ook[2];
    float wv[2];
    float4 av[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int it = tid + 256 * h;
        const int rb = it / L, x = it - (it / L) * L;
        ook[h] = row0 + rb < rows && x < N1;
        oi[h] = (long long)min(row0 + rb, rows - 1) * N1 + min(x, N1 - 1);
        ol[h] = rb * L + (x >> 1);
        wv[h] = src_mode > 0 ? wc[oi[h]] : 1.f;
        av[h] = src_mode == 2 ? wstat[oi[h]] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    // a finished controller turns the kernel into a no-op; the flag is read
    // after the data loads are issued, so its round trip overlaps theirs
    if (ctrl && ctrl->done) return;
    load_twiddles<2 * L, 256>(tl, tw, tid);
    __syncthreads();
    // Z_k = E_k + i O_k with E_k = X_k + conj X_{L-k},
    // O_k = (X_k - conj X_{L-k}) W^-k: the length-L inverse then yields
    // P1 * (a_2n + i a_2n+1)
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int it = tid + i * 256;
        const int rb = it / L, k = it - (it / L) * L;
        const float2 wi = twiddle<1>(tl, k);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 e = cadd(xk[i][c], xc[i][c]);
            const float2 o = cmul(csub(xk[i][c], xc[i][c]), wi);
            s[(c * RB + rb) * L + k] = make_float2(e.x - o.y, e.y + o.x);
        }
    }
    __syncthreads();
    lds_fft<L, 1, NP, 256, false, 2 * L>(s, tl, tid);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        if (!ook[h]) continue;
        const bool odd = (tid + 256 * h) & 1;   // L is even: the cell's parity
        float v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float2 e = s[c * RB * L + ol[h]];
            v[c] = odd ? e.y : e.x;
        }
        if (src_mode == 0) {
#pragma unroll
            for (int c = 0; c < 3; ++c) hd[c * nc + oi[h]] = v[c];
        } else {
            // the node kernel's source, one float4 per cell
            reinterpret_cast<float4 *>(hd)[oi[h]] =
                make_float4(wv[h] * v[0] + av[h].x, wv[h] * v[1] + av[h].y, wv[h] * v[2] + av[h].z, av[h].w);
        }
    }
}

template <int L>
__global__ void __launch_bounds__(256)
k_xinv(const float2 *__restrict__ spec, float *__restrict__ hd, const float2 *__restrict__ tw,
       int N1, int N2, int N3, int P2, int KP, const float *__restrict__ wc,
       const float4 *__restrict__ wstat, int src_mode, const Ctrl *__restrict__ ctrl) {
    xinv_body<L>(spec, hd, tw, N1, N2, N3, P2, KP, wc, wstat, src_mode, ctrl, blockIdx.x);
}

// ----------------------------------------- y pass, register FFT form
// NPB columns per block, T threads per column (fft2 split of L).  Forward:
// the N2 <= L / 2 data rows in, all L rows out.  Inverse: all L rows in, the
// N2 data rows out.
template <int L, int DIR, int SH>
__device__ __forceinline__ void ypass_body(float2 *__restrict__ spec, const float2 *__restrict__ tw, int N3,
                                           int N2, int K1, int KP, const Ctrl *__restrict__ ctrl, int bx,
                                           int comp) {
    constexpr int L1 = fft2_l1(L), L2 = L / L1, TT = fft2_threads(L);
    constexpr int NPB = (256 / TT) >> SH, E = L / TT, NT = NPB * TT;   // 2^-SH of the widest block
    static_assert(NPB >= 1, "block width");
    __shared__ float2 sh[TT > 1 ? L * NPB : 1];
    __shared__ float2 tl[L];
    const int tid = threadIdx.x, b = tid % NPB, j = tid / NPB;
    const int col = bx * NPB + b;
    const int zc = col / KP, kx = col - zc * KP;
    const bool inrow = col < N3 * KP, valid = inrow && kx < K1;
    // 32-bit byte offsets within one component (N3 P2 KP complex < 4 GiB);
    // pad lanes (K1 <= kx < KP) read their own zeroed column, past-the-end
    // lanes column 0
    float2 *cb = spec + (long long)comp * N3 * L * KP;
    const unsigned oc = inrow ? 8u * ((unsigned)zc * (unsigned)(L * KP) + (unsigned)kx) : 0u;
    const unsigned rs = 8u * (unsigned)KP;   // row stride
    float2 v[1][E];
    if constexpr (DIR < 0) {
        // rows (j + T a) + L1 n2; only n2 < L2 / 2 can hold data
        constexpr int A = L1 / TT;
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int n2 = 0; n2 < L2; ++n2) {
                float2 x = make_float2(0.f, 0.f);
                if (n2 < L2 / 2) {
                    const int y = j + TT * a + L1 * n2;
                    x = keep(ldo(cb, oc + (unsigned)min(y, N2 - 1) * rs), valid && y < N2);
                }
                v[0][a * L2 + n2] = x;
            }
        if (ctrl && ctrl->done) return;   // read after the loads are issued
        load_twiddles_full<L, NT>(tl, tw, tid);
        fft2<L1, L2, -1, 1, NPB, E, true, false>(v, sh, tl, j, b);
        if (!valid) return;
        // rows (j + T q) + L2 k1
        constexpr int Q = L2 / TT;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1) sto(cb, oc + (unsigned)(j + TT * q + L2 * k1) * rs, v[0][q * L1 + k1]);
    } else {
        // rows (j + T q) + L2 k1 in (the forward output layout)
        constexpr int Q = L2 / TT;
#pragma unroll
        for (int q = 0; q < Q; ++q)
#pragma unroll
            for (int k1 = 0; k1 < L1; ++k1)
                v[0][q * L1 + k1] = keep(ldo(cb, oc + (unsigned)(j + TT * q + L2 * k1) * rs), valid);
        if (ctrl && ctrl->done) return;   // read after the loads are issued
        load_twiddles_full<L, NT>(tl, tw, tid);
        fft2<L2, L1, 1, 1, NPB, E, false, true>(v, sh, tl, j, b);
        if (!valid) return;
        // rows (j + T a) + L1 n2 out; only n2 < L2 / 2 can be data rows
        constexpr int A = L1 / TT;
#pragma unroll
        for (int a = 0; a < A; ++a)
#pragma unroll
            for (int n2 = 0; n2 < L2 / 2; ++n2) {
                const int y = j + TT * a + L1 * n2;
                if (y < N2) sto(cb, oc + (unsigned)y * rs, v[0][a * L2 + n2]);
            }
    }
}

template <int L, int DIR, int SH>
__global__ void __launch_bounds__(256)
k_ypass_r(float2 *__restrict__ spec, const float2 *__restrict__ tw, int N3, int N2, int K1, int KP,
          const Ctrl *__restrict__ ctrl) {
    ypass_body<L, DIR, SH>(spec, tw, N3, N2, K1, KP, ctrl, blockIdx.x, blockIdx.y);
}

// ------------------------------------------- k-space product of one element
struct Tensor6 {
    float xx, yy, zz, xy, xz, yz;
};

__device__ __forceinline__ Tensor6 tensor_load(const float *__restrict__ T, long long tstride,
                                               long long tidx, float sy, bool full3d) {
    Tensor6 N;
    N.xx = T[tidx];
    N.yy = T[tstride + tidx];
    N.zz = T[2 * tstride + tidx];
    N.xy = sy * T[3 * tstride + tidx];
    N.xz = full3d ? T[4 * tstride + tidx] : 0.f;
    N.yz = full3d ? sy * T[5 * tstride + tidx] : 0.f;
    return N;
}

// the same with 32-bit byte offsets from per-component bases (off = 4 tidx)
__device__ __forceinline__ Tensor6 tensor_load32(const float *__restrict__ T, long long tstride,
                                                 unsigned off, float sy) {
    Tensor6 N;
    N.xx = ldo(T, off);
    N.yy = ldo(T + tstride, off);
    N.zz = ldo(T + 2 * tstride, off);
    N.xy = sy * ldo(T + 3 * tstride, off);
    N.xz = ldo(T + 4 * tstride, off);
    N.yz = sy * ldo(T + 5 * tstride, off);
    return N;
}

// H^ = -N^ M^ in place; sz flips the components odd along the fused axis
__device__ __forceinline__ void tensor_apply(const Tensor6 &N, float sz, float2 &mx, float2 &my, float2 &mz) {
    const float xz = sz * N.xz, yz = sz * N.yz;
    const float2 hx = make_float2(-(N.xx * mx.x + N.xy * my.x + xz * mz.x), -(N.xx * mx.y + N.xy * my.y + xz * mz.y));
    const float2 hy = make_float2(-(N.xy * mx.x + N.yy * my.x + yz * mz.x), -(N.xy * mx.y + N.yy * my.y + yz * mz.y));
    const float2 hz = make_float2(-(xz * mx.x + yz * my.x + N.zz * mz.x), -(xz * mx.y + yz * my.y + N.zz * mz.y));
    mx = hx;
    my = hy;
    mz = hz;
}

// ------------------------------------------- z forward + product + z inverse
// columns (ky < P2, kx < K1) at pitch KP are contiguous; elements along z at stride P2 KP
template <int L, int TB>
__global__ void __launch_bounds__(256)
k_zconv(float2 *__restrict__ spec, const float *__restrict__ T, const float2 *__restrict__ tw,
        int N3, int P2, int K1, int KP, int P2h, int P3h, const Ctrl *__restrict__ ctrl) {
    constexpr int NP = 3 * TB;
    __shared__ float2 s[(L + 1) * NP];   // + one spare row for masked lanes
    __shared__ float2 tl[L / 2 + 1];
    const int tid = threadIdx.x;
    const long long plane = (long long)P2 * KP;
    const int ncols = P2 * KP;
    // neighbouring column tiles on one XCD: a tile is narrower than a cache
    // line, and the tiles next to it read the rest of each line from L2
    const int col0 = (int)xcd_block(blockIdx.x, gridDim.x) * TB;
    // tiles of <= 16 columns never cross a ky row (KP is a multiple of 16)
    const int kx0 = col0 % KP;
    auto valid = [&](int b) {
        const int col = col0 + b;
        const int kx = TB <= 16 ? kx0 + b : col % KP;
        return col < ncols && kx < K1;
    };
    // planes past N3 and pad columns: clamped reads zeroed by a select
    static_assert((L * NP) % 256 == 0, "whole iterations");
    constexpr int NI = L * NP / 256;
    float2 v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int it = tid + i * 256;
        const int p = it % NP, e = it / NP;
        const int c = p / TB, b = p - (p / TB) * TB;
        const bool ok = e < N3 && valid(b);
        const int col = valid(b) ? col0 + b : col0 - kx0;
        const float2 t = spec[((long long)c * N3 + min(e, N3 - 1)) * plane + col];
        v[i] = keep(t, ok);
    }
    // the tensor entries this thread applies after the forward transform,
    // fetched now so their latency hides behind the FFT
    const long long tstride = (long long)P3h * P2h * KP;
    constexpr int NT = ((L / 2 + 1) * TB + 255) / 256;
    Tensor6 Nt[NT];
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int it = tid + i * 256;
        const int b = it % TB, kzr = it / TB;
        const bool ok = valid(b) && kzr <= L / 2;
        const int col = ok ? col0 + b : col0 - kx0;
        const int ky = col / KP, kx = col - (col / KP) * KP;
        const bool fy = ky > P2 / 2;
        const int kyr = fy ? P2 - ky : ky;
        Nt[i] = tensor_load(T, tstride, ((long long)(ok ? kzr : 0) * P2h + kyr) * KP + kx, fy ? -1.f : 1.f, true);
    }
    // a finished controller turns the kernel into a no-op; the flag is read
    // after the data loads are issued, so its round trip overlaps theirs
    if (ctrl && ctrl->done) return;
    load_twiddles<L, 256>(tl, tw, tid);
#pragma unroll
    for (int i = 0; i < NI; ++i) s[tid + i * 256] = v[i];   // = s[e * NP + p]
    __syncthreads();
    lds_fft<L, -1, NP, 256, true, L>(s, tl, tid);
    // kz and L - kz share the stored tensor entry (xz, yz flip sign): one read
    // serves both.  Branch-free: lanes without a valid (column, kz) use a
    // clamped entry and write their product into the spare row s[L * NP ..]
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int it = tid + i * 256;
        const int b = it % TB, kzr = it / TB;
        const bool ok = valid(b) && kzr <= L / 2;
        const int kzc = ok ? kzr : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int kz = h == 0 ? kzc : (L - kzc) & (L - 1);
            const bool wr = ok && (h == 0 || (kzr != 0 && kzr != L / 2));
            const int row = wr ? kz * NP : L * NP;
            float2 mx = s[kz * NP + b], my = s[kz * NP + TB + b], mz = s[kz * NP + 2 * TB + b];
            tensor_apply(Nt[i], h == 0 ? 1.f : -1.f, mx, my, mz);
            s[row + b] = mx;
            s[row + TB + b] = my;
            s[row + 2 * TB + b] = mz;
        }
    }
    __syncthreads();
    lds_fft<L, 1, NP, 256, true, L>(s, tl, tid);
    for (int it = tid; it < N3 * NP; it += 256) {
        const int p = it % NP, e = it / NP;
        const int c = p / TB, b = p - (p / TB) * TB;
        const int col = col0 + b;
        if (valid(b)) spec[((long long)c * N3 + e) * plane + col] = s[e * NP + p];
    }
}

// ----------------------- z forward + product + z inverse, register FFT form
// NPB columns per block, T threads per column (fft2 split of L), all three
// components of a column in the same thread, so the product with the tensor
// happens in registers between the forward and the inverse transform.  Only
// z < L / 2 can hold data (P3 >= 2 N3), so half of the inputs are known zeros
// and half of the outputs are never stored.
template <int L, int SH>
__device__ __forceinline__ void zconv_r_body(float2 *__restrict__ spec, const float *__restrict__ T,
                                             const float2 *__restrict__ tw, int N3, int P2, int K1, int KP,
                                             int P2h, int P3h, const Ctrl *__restrict__ ctrl, int lblock) {
    constexpr int L1 = fft2_l1(L), L2 = L / L1, TT = fft2_threads(L);
    constexpr int NPB = (256 / TT) >> SH, E = L / TT, A = L1 / TT, NT = NPB * TT;
    static_assert(NPB >= 1, "block width");
    constexpr int NCX = E <= 8 ? 3 : 1;   // components per LDS exchange
    __shared__ float2 sh[TT > 1 ? NCX * L * NPB : 1];
    __shared__ float2 tl[L];
    const int tid = threadIdx.x, b = tid % NPB, j = tid / NPB;
    // columns in mirror order: ky rows 0, 1, P2-1, 2, P2-2, ..., P2/2 (rows ky
    // and P2-ky read the same stored tensor entries), blocks in contiguous
    // ranges per XCD, so a row's mirror finds the tensor in the same L2
    const int pos = lblock * NPB + b;
    const int slot = pos / KP, kxp = pos - slot * KP;
    const int kyp = slot == 0 ? 0 : slot >= P2 - 1 ? P2 / 2 : (slot & 1) ? (slot + 1) / 2 : P2 - (slot + 1) / 2;
    const int col = kyp * KP + kxp;
    const bool inrange = pos < P2 * KP, valid = inrange && kxp < K1;
    // pad lanes (K1 <= kx < KP) read their own zeroed column, past-the-end
    // lanes column 0
    const int colc = inrange ? col : 0;
    const long long plane = (long long)P2 * KP;
    // inputs z = (j + T a) + L1 n2, nonzero only for n2 < L2 / 2; 32-bit byte
    // offsets within one component (N3 P2 KP complex < 4 GiB)
    float2 *sp[3] = {spec, spec + (long long)N3 * plane, spec + 2LL * N3 * plane};
    float2 v[3][E];
#pragma unroll
    for (int a = 0; a < A; ++a)
#pragma unroll
        for (int n2 = 0; n2 < L2; ++n2) {
            if (n2 < L2 / 2) {
                const int z = j + TT * a + L1 * n2;
                const unsigned off = 8u * ((unsigned)min(z, N3 - 1) * (unsigned)plane + (unsigned)colc);
                const bool ok = valid && z < N3;
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c][a * L2 + n2] = keep(ldo(sp[c], off), ok);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c][a * L2 + n2] = make_float2(0.f, 0.f);
            }
        }
    // tensor entries of this thread's frequencies kz = (j + T q) + L2 k1
    // (kz and L - kz share the stored entry, xz and yz change sign)
    const int ky = colc / KP, kx = colc - ky * KP;
    const bool fy = ky > P2 / 2;
    const int kyr = fy ? P2 - ky : ky;
    const long long tstride = (long long)P3h * P2h * KP;
    auto tensor_at = [&](int i) {
        const int kz = j + TT * (i / L1) + L2 * (i % L1);
        const int kzr = kz <= L / 2 ? kz : L - kz;
        return tensor_load32(T, tstride, 4u * (((unsigned)kzr * (unsigned)P2h + (unsigned)kyr) * (unsigned)KP + (unsigned)kx),
                             fy ? -1.f : 1.f);
    };
    auto apply = [&](int i, const Tensor6 &N) {
        const int kz = j + TT * (i / L1) + L2 * (i % L1);
        tensor_apply(N, kz <= L / 2 ? 1.f : -1.f, v[0][i], v[1][i], v[2][i]);
    };
    // The tensor entries are loaded where they are applied, after the forward
    // transform: fetching all E of them up front (to hide their latency
    // behind the transform) costs 24 VGPRs and measured 7% slower at L = 64.
    // a finished controller turns the kernel into a no-op; the flag is read
    // after the data loads are issued, so its round trip overlaps theirs
    if (ctrl && ctrl->done) return;
    load_twiddles_full<L, NT>(tl, tw, tid);
    if constexpr (NCX == 3) {
        fft2<L1, L2, -1, 3, NPB, E, true, false>(v, sh, tl, j, b);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            fft2<L1, L2, -1, 1, NPB, E, true, false>(*reinterpret_cast<float2(*)[1][E]>(&v[c]), sh, tl, j, b);
    }
#pragma unroll
    for (int i = 0; i < E; ++i) apply(i, tensor_at(i));
    if constexpr (NCX == 3) {
        fft2<L2, L1, 1, 3, NPB, E, false, true>(v, sh, tl, j, b);
    } else {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            fft2<L2, L1, 1, 1, NPB, E, false, true>(*reinterpret_cast<float2(*)[1][E]>(&v[c]), sh, tl, j, b);
    }
    if (!valid) return;
#pragma unroll
    for (int a = 0; a < A; ++a)
#pragma unroll
        for (int n2 = 0; n2 < L2 / 2; ++n2) {
            const int z = j + TT * a + L1 * n2;
            const unsigned off = 8u * ((unsigned)z * (unsigned)plane + (unsigned)col);
            if (z < N3)
#pragma unroll
                for (int c = 0; c < 3; ++c) sto(sp[c], off, v[c][a * L2 + n2]);
        }
}

template <int L, int SH>
__global__ void __launch_bounds__(256)
k_zconv_r(float2 *__restrict__ spec, const float *__restrict__ T, const float2 *__restrict__ tw,
          int N3, int P2, int K1, int KP, int P2h, int P3h, const Ctrl *__restrict__ ctrl) {
    zconv_r_body<L, SH>(spec, T, tw, N3, P2, K1, KP, P2h, P3h, ctrl, (int)xcd_block(blockIdx.x, gridDim.x));
}

// ------------------------------------ y forward + product + y inverse (N3 = 1)
// NTH threads per block (yconv_threads): the long columns of large films
// are few (K1 = P1/2 + 1 of them, one per block), so each gets more threads
// (512 at L = 1024: 9% faster than 256; 1024 gained nothing)
template <int L, int TB, int NTH>
__device__ __forceinline__ void yconv_body(float2 *__restrict__ spec, const float *__restrict__ T,
                                           const float2 *__restrict__ tw, int N2, int K1, int KP, int P2h,
                                           const Ctrl *__restrict__ ctrl, int lblock) {
    constexpr int NP = 3 * TB;
    __shared__ float2 s[(L + 1) * NP];   // + one spare row for masked lanes
    __shared__ float2 tl[L / 2 + 1];
    const int tid = threadIdx.x;
    const long long cstride = (long long)L * KP;
    // neighbouring column tiles on one XCD: a tile is narrower than a cache
    // line, and the tiles next to it read the rest of each line from L2
    const int col0 = lblock * TB;
    static_assert((L * NP) % NTH == 0, "whole iterations");
    constexpr int NI = L * NP / NTH;
    float2 v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int it = tid + i * NTH;
        const int p = it % NP, e = it / NP;
        const int c = p / TB, b = p - (p / TB) * TB;
        const int col = col0 + b;
        const float2 t = spec[c * cstride + (long long)min(e, N2 - 1) * KP + min(col, K1 - 1)];
        v[i] = keep(t, col < K1 && e < N2);
    }
    const long long tstride = (long long)P2h * KP;
    constexpr int NT = ((L / 2 + 1) * TB + NTH - 1) / NTH;
    Tensor6 Nt[NT];   // fetched now, applied after the forward transform
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int it = tid + i * NTH;
        const int b = it % TB, kyr = it / TB;
        const bool ok = col0 + b < K1 && kyr <= L / 2;
        Nt[i] = tensor_load(T, tstride, (long long)(ok ? kyr : 0) * KP + min(col0 + b, K1 - 1), 1.f, false);
    }
    // a finished controller turns the kernel into a no-op; the flag is read
    // after the data loads are issued, so its round trip overlaps theirs
    if (ctrl && ctrl->done) return;
    load_twiddles<L, NTH>(tl, tw, tid);
#pragma unroll
    for (int i = 0; i < NI; ++i) s[tid + i * NTH] = v[i];
    __syncthreads();
    lds_fft<L, -1, NP, NTH, true, L>(s, tl, tid);
    // ky and L - ky share the stored tensor entry (xy flips sign)
#pragma unroll
    for (int i = 0; i < NT; ++i) {
        const int it = tid + i * NTH;
        const int b = it % TB, kyr = it / TB;
        const bool ok = col0 + b < K1 && kyr <= L / 2;
        const int kyc = ok ? kyr : 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ky = h == 0 ? kyc : (L - kyc) & (L - 1);
            const bool wr = ok && (h == 0 || (kyr != 0 && kyr != L / 2));
            const int row = wr ? ky * NP : L * NP;
            Tensor6 Nh = Nt[i];
            if (h == 1) Nh.xy = -Nh.xy;
            float2 mx = s[ky * NP + b], my = s[ky * NP + TB + b], mz = s[ky * NP + 2 * TB + b];
            tensor_apply(Nh, 1.f, mx, my, mz);
            s[row + b] = mx;
            s[row + TB + b] = my;
            s[row + 2 * TB + b] = mz;
        }
    }
    __syncthreads();
    lds_fft<L, 1, NP, NTH, true, L>(s, tl, tid);
    for (int it = tid; it < N2 * NP; it += NTH) {
        const int p = it % NP, e = it / NP;
        const int c = p / TB, b = p - (p / TB) * TB;
        const int col = col0 + b;
        if (col < K1) spec[c * cstride + (long long)e * KP + col] = s[e * NP + p];
    }
}

__host__ __device__ constexpr int yconv_threads(int L) { return L >= 1024 ? 512 : 256; }

template <int L, int TB>
__global__ void __launch_bounds__(yconv_threads(L))
k_yconv(float2 *__restrict__ spec, const float *__restrict__ T, const float2 *__restrict__ tw,
        int N2, int K1, int KP, int P2h, const Ctrl *__restrict__ ctrl) {
    yconv_body<L, TB, yconv_threads(L)>(spec, T, tw, N2, K1, KP, P2h, ctrl, (int)xcd_block(blockIdx.x, gridDim.x));
}

// --------------------------------------------------------------- dispatch
// column tiles of the LDS-sweep convolutions: three components per block,
// 3 L TB <= 4096 elements
__host__ __device__ constexpr int tb_triple(int L) { return L <= 16 ? 64 : 1024 / L; }

template <int L>
static void launch_x_fwd(nm_mesh *m, const float *mag, const float2 *tw, const Ctrl *ctrl) {
    constexpr int RB = x_rows_per_block(L);
    NM_LAUNCH(m, NM_PROF_XFWD, (k_xfwd<L>), dim3((m->N2 + RB - 1) / RB, m->N3), dim3(256), 0, mag,
              m->Ms, m->spec, tw, m->N1, m->N2, m->N3, m->NZ, m->P2, m->KP, ctrl);
}
template <int L>
static void launch_x_inv(nm_mesh *m, const float2 *tw, const Ctrl *ctrl, int src_mode) {
    constexpr int RB = x_rows_per_block(L);
    const int rows = m->N2 * m->N3;
    NM_LAUNCH(m, NM_PROF_XINV, (k_xinv<L>), dim3((rows + RB - 1) / RB), dim3(256), 0, m->spec, m->hd,
              tw, m->N1, m->N2, m->N3, m->P2, m->KP, m->wc, m->wstat, src_mode, ctrl);
}
// block width of the register-FFT passes: the widest column tile shifted
// right by SH (0 widest, 1 half, 2 quarter), chosen per mesh by tune_passes
template <int L, int DIR, int SH>
static void launch_y_sh(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    constexpr int TT = fft2_threads(L), NPB = (256 / TT) >> SH;
    const int ncols = m->N3 * m->KP;
    NM_LAUNCH(m, DIR < 0 ? NM_PROF_YFWD : NM_PROF_YINV, (k_ypass_r<L, DIR, SH>),
              dim3((ncols + NPB - 1) / NPB, 3), dim3(NPB * TT), 0, m->spec, tw, m->N3, m->N2, m->K1, m->KP, ctrl);
}
template <int L, int DIR>
static void launch_y(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    switch (m->tune_y) {
        case 1: if constexpr ((256 / fft2_threads(L)) >= 2) { launch_y_sh<L, DIR, 1>(m, tw, ctrl); return; } break;
        case 2: if constexpr ((256 / fft2_threads(L)) >= 4) { launch_y_sh<L, DIR, 2>(m, tw, ctrl); return; } break;
        default: break;
    }
    launch_y_sh<L, DIR, 0>(m, tw, ctrl);
}
template <int L, int SH>
static void launch_zconv_sh(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    constexpr int TT = fft2_threads(L), NPB = (256 / TT) >> SH;
    const int ncols = m->P2 * m->KP;
    NM_LAUNCH(m, NM_PROF_CONV, (k_zconv_r<L, SH>), dim3((ncols + NPB - 1) / NPB), dim3(NPB * TT), 0, m->spec,
              m->tensor, tw, m->N3, m->P2, m->K1, m->KP, m->P2h, m->P3h, ctrl);
}
template <int L>
static void launch_zconv(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    if constexpr (L <= 256) {
        switch (m->tune_z) {
            case 1: if constexpr ((256 / fft2_threads(L)) >= 2) { launch_zconv_sh<L, 1>(m, tw, ctrl); return; } break;
            case 2: if constexpr ((256 / fft2_threads(L)) >= 4) { launch_zconv_sh<L, 2>(m, tw, ctrl); return; } break;
            default: break;
        }
        launch_zconv_sh<L, 0>(m, tw, ctrl);
    } else {
        constexpr int TB = tb_triple(L);
        const int ncols = m->P2 * m->KP;
        NM_LAUNCH(m, NM_PROF_CONV, (k_zconv<L, TB>), dim3((ncols + TB - 1) / TB), dim3(256), 0, m->spec,
                  m->tensor, tw, m->N3, m->P2, m->K1, m->KP, m->P2h, m->P3h, ctrl);
    }
}
template <int L>
static void launch_yconv(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    constexpr int TB = tb_triple(L);
    NM_LAUNCH(m, NM_PROF_CONV, (k_yconv<L, TB>), dim3((m->K1 + TB - 1) / TB), dim3(yconv_threads(L)), 0, m->spec,
              m->tensor, tw, m->N2, m->K1, m->KP, m->P2h, ctrl);
}

// row passes: half lengths 2..512 (P1 = 4..1024); column passes: 4..1024
// (n >= 2 cells along y, and along z whenever the z pass runs)
#define NM_DISPATCH_ROW(LEN, FN, ...)                        \
    switch (LEN) {                                           \
        case 2: FN<2>(__VA_ARGS__); break;                   \
        case 4: FN<4>(__VA_ARGS__); break;                   \
        case 8: FN<8>(__VA_ARGS__); break;                   \
        case 16: FN<16>(__VA_ARGS__); break;                 \
        case 32: FN<32>(__VA_ARGS__); break;                 \
        case 64: FN<64>(__VA_ARGS__); break;                 \
        case 128: FN<128>(__VA_ARGS__); break;               \
        case 256: FN<256>(__VA_ARGS__); break;               \
        case 512: FN<512>(__VA_ARGS__); break;               \
        default: return hipErrorInvalidValue;                \
    }
#define NM_DISPATCH_COL(LEN, FN, ...)                        \
    switch (LEN) {                                           \
        case 4: FN<4>(__VA_ARGS__); break;                   \
        case 8: FN<8>(__VA_ARGS__); break;                   \
        case 16: FN<16>(__VA_ARGS__); break;                 \
        case 32: FN<32>(__VA_ARGS__); break;                 \
        case 64: FN<64>(__VA_ARGS__); break;                 \
        case 128: FN<128>(__VA_ARGS__); break;               \
        case 256: FN<256>(__VA_ARGS__); break;               \
        case 512: FN<512>(__VA_ARGS__); break;               \
        case 1024: FN<1024>(__VA_ARGS__); break;             \
        default: return hipErrorInvalidValue;                \
    }

template <int L>
static void launch_y_fwd(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    launch_y<L, -1>(m, tw, ctrl);
}
template <int L>
static void launch_y_inv(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    launch_y<L, 1>(m, tw, ctrl);
}

static hipError_t demag_pipeline(nm_mesh *m, const float *mag, const Ctrl *ctrl, int src_mode) {
    const float2 *tw = twiddles(m->device);
    if (!tw) return hipErrorOutOfMemory;
    const int L1 = m->P1 / 2;
    NM_DISPATCH_ROW(L1, launch_x_fwd, m, mag, tw, ctrl);
    if (m->N3 > 1) {
        NM_DISPATCH_COL(m->P2, launch_y_fwd, m, tw, ctrl);
        NM_DISPATCH_COL(m->P3, launch_zconv, m, tw, ctrl);
        NM_DISPATCH_COL(m->P2, launch_y_inv, m, tw, ctrl);
    } else {
        NM_DISPATCH_COL(m->P2, launch_yconv, m, tw, ctrl);
    }
    NM_DISPATCH_ROW(L1, launch_x_inv, m, tw, ctrl, src_mode);
    return hipGetLastError();
}

// ------------------------------------------------------------ tile tuner
// Block widths of the register-FFT passes, chosen per padded shape by timing
// every width on the mesh itself (a warm-up and 5 launches, three times
// each) and cached per (P1, P2, P3, N2, N3, device).  Small meshes run
// only a few dozen blocks per pass, where narrower blocks finish sooner;
// large ones keep the widest.  Every width computes each column identically,
// so the choice never changes results.
namespace {
struct TuneKey {
    int p1, p2, p3, n2, n3, dev;
    bool operator<(const TuneKey &o) const {
        return std::tie(p1, p2, p3, n2, n3, dev) < std::tie(o.p1, o.p2, o.p3, o.n2, o.n3, o.dev);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tune;

template <int L>
void launch_y_pair(nm_mesh *m, const float2 *tw, const Ctrl *ctrl) {
    launch_y<L, -1>(m, tw, ctrl);
    launch_y<L, 1>(m, tw, ctrl);
}

}  // namespace

int tile_widths(int L) {   // how many of the shifts 0, 1, 2 exist for length L
    const int npb = 256 / fft2_threads_host(L);
    return npb >= 4 ? 3 : npb >= 2 ? 2 : 1;
}

hipError_t tune_passes(nm_mesh *m) {
    m->tune_y = m->tune_z = 0;
    if (m->N3 == 1) return hipSuccess;   // films use the fused y convolution
    const TuneKey key{m->P1, m->P2, m->P3, m->N2, m->N3, m->device};
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            m->tune_y = it->second.first;
            m->tune_z = it->second.second;
            return hipSuccess;
        }
    }
    const float2 *tw = twiddles(m->device);
    if (!tw) return hipErrorOutOfMemory;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    auto time_it = [&](auto run, float *ms) -> hipError_t {
        hipError_t r = run();   // warm-up
        if (r == hipSuccess) r = hipEventRecord(e0, m->stream);
        for (int k = 0; k < 5 && r == hipSuccess; ++k) r = run();
        if (r == hipSuccess) r = hipEventRecord(e1, m->stream);
        if (r == hipSuccess) r = hipEventSynchronize(e1);
        if (r == hipSuccess) r = hipEventElapsedTime(ms, e0, e1);
        return r;
    };
    // each width timed three times, interleaved, keeping its fastest; the
    // widest tile wins unless a narrower one is at least 5% faster (single
    // timings of a few launches are noisy, and a narrower tile that wins by
    // noise in isolation can lose inside the pipeline)
    auto pick = [&](int nw, auto run_v, int *best) -> hipError_t {
        float t[3] = {1e30f, 1e30f, 1e30f};
        hipError_t r = hipSuccess;
        for (int rep = 0; rep < 3 && r == hipSuccess; ++rep)
            for (int v = 0; v < nw && r == hipSuccess; ++v) {
                float ms = 0.f;
                r = time_it([&]() -> hipError_t { return run_v(v); }, &ms);
                if (r == hipSuccess) t[v] = fminf(t[v], ms);
            }
        int b = 0;
        for (int v = 1; v < nw; ++v)
            if (t[v] < 0.95f * t[b]) b = v;
        *best = b;
        return r;
    };
    int best_y = 0, best_z = 0;
    if (e == hipSuccess)
        e = pick(tile_widths(m->P2), [&](int v) -> hipError_t {
            m->tune_y = v;
            NM_DISPATCH_COL(m->P2, launch_y_pair, m, tw, nullptr);
            return hipGetLastError();
        }, &best_y);
    if (e == hipSuccess && m->P3 <= 256)
        e = pick(tile_widths(m->P3), [&](int v) -> hipError_t {
            m->tune_z = v;
            NM_DISPATCH_COL(m->P3, launch_zconv, m, tw, nullptr);
            return hipGetLastError();
        }, &best_z);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    m->tune_y = best_y;
    m->tune_z = best_z;
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {best_y, best_z};
    return hipSuccess;
}

// ------------------------------------------------------ batched launches
// One launch per pass covers every slot of a batch group (grid z = slot);
// grids cover the largest mesh of the class, and blocks past a slot's own
// rows or columns return before any work.  Each block runs the single-mesh
// kernel's code on its slot's buffers, so results do not depend on the group.
template <int L>
__global__ void __launch_bounds__(256) k_xfwd_b(const BatchSlot *__restrict__ slots, int stage,
                                                const float2 *__restrict__ tw) {
    const BatchSlot &d = slots[blockIdx.z];
    constexpr int RB = x_rows_per_block(L);
    int bx, by;
    xfwd_block<L>(bx, by);
    if (!d.active || bx * RB >= d.N2 || by >= d.N3) return;
    xfwd_body<L>(d.stage_in[stage], d.Ms, d.spec, tw, d.N1, d.N2, d.N3, d.NZ, d.P2, d.KP, d.ctrl, bx, by);
}
template <int L>
__global__ void __launch_bounds__(256) k_xinv_b(const BatchSlot *__restrict__ slots, const float2 *__restrict__ tw) {
    const BatchSlot &d = slots[blockIdx.z];
    constexpr int RB = x_rows_per_block(L);
    if (!d.active || (int)blockIdx.x * RB >= d.N2 * d.N3) return;
    xinv_body<L>(d.spec, d.hd, tw, d.N1, d.N2, d.N3, d.P2, d.KP, d.wc, d.wstat, d.src_mode, d.ctrl, blockIdx.x);
}
template <int L, int DIR, int SH>
__global__ void __launch_bounds__(256) k_ypass_b(const BatchSlot *__restrict__ slots, const float2 *__restrict__ tw) {
    const BatchSlot &d = slots[blockIdx.z];
    constexpr int NPB = (256 / fft2_threads(L)) >> SH;
    if (!d.active || (int)blockIdx.x * NPB >= d.N3 * d.KP) return;
    ypass_body<L, DIR, SH>(d.spec, tw, d.N3, d.N2, d.K1, d.KP, d.ctrl, blockIdx.x, blockIdx.y);
}
template <int L, int SH>
__global__ void __launch_bounds__(256) k_zconv_b(const BatchSlot *__restrict__ slots, const float2 *__restrict__ tw) {
    const BatchSlot &d = slots[blockIdx.z];
    if (!d.active) return;
    zconv_r_body<L, SH>(d.spec, d.tensor, tw, d.N3, d.P2, d.K1, d.KP, d.P2h, d.P3h, d.ctrl,
                        (int)xcd_block(blockIdx.x, gridDim.x));
}
template <int L, int TB>
__global__ void __launch_bounds__(yconv_threads(L)) k_yconv_b(const BatchSlot *__restrict__ slots,
                                                              const float2 *__restrict__ tw) {
    const BatchSlot &d = slots[blockIdx.z];
    if (!d.active) return;
    yconv_body<L, TB, yconv_threads(L)>(d.spec, d.tensor, tw, d.N2, d.K1, d.KP, d.P2h, d.ctrl,
                                        (int)xcd_block(blockIdx.x, gridDim.x));
}
namespace {
struct BatchLaunch {
    const BatchClass &bc;
    const BatchSlot *slots;
    int cap, stage;
    hipStream_t st;
    const float2 *tw;
    int KP() const { return ((bc.P1 / 2 + 1) + 15) / 16 * 16; }
};

template <int L>
void launch_xfwd_bt(const BatchLaunch &b) {
    constexpr int RB = x_rows_per_block(L);
    hipLaunchKernelGGL((k_xfwd_b<L>), dim3((b.bc.gN2 + RB - 1) / RB, b.bc.gN3, b.cap), dim3(256), 0, b.st, b.slots,
                       b.stage, b.tw);
}
template <int L>
void launch_xinv_bt(const BatchLaunch &b) {
    constexpr int RB = x_rows_per_block(L);
    const int rows = b.bc.gN2 * b.bc.gN3;
    hipLaunchKernelGGL((k_xinv_b<L>), dim3((rows + RB - 1) / RB, 1, b.cap), dim3(256), 0, b.st, b.slots, b.tw);
}
template <int L, int DIR, int SH>
void launch_ypass_bsh(const BatchLaunch &b) {
    constexpr int TT = fft2_threads(L), NPB = (256 / TT) >> SH;
    const int ncols = b.bc.gN3 * b.KP();
    hipLaunchKernelGGL((k_ypass_b<L, DIR, SH>), dim3((ncols + NPB - 1) / NPB, 3, b.cap), dim3(NPB * TT), 0, b.st,
                       b.slots, b.tw);
}
template <int L, int DIR>
void launch_ypass_bt(const BatchLaunch &b) {
    switch (b.bc.tune_y) {
        case 1: if constexpr ((256 / fft2_threads(L)) >= 2) { launch_ypass_bsh<L, DIR, 1>(b); return; } break;
        case 2: if constexpr ((256 / fft2_threads(L)) >= 4) { launch_ypass_bsh<L, DIR, 2>(b); return; } break;
        default: break;
    }
    launch_ypass_bsh<L, DIR, 0>(b);
}
template <int L>
void launch_yfwd_bt(const BatchLaunch &b) { launch_ypass_bt<L, -1>(b); }
template <int L>
void launch_yinv_bt(const BatchLaunch &b) { launch_ypass_bt<L, 1>(b); }
template <int L, int SH>
void launch_zconv_bsh(const BatchLaunch &b) {
    constexpr int TT = fft2_threads(L), NPB = (256 / TT) >> SH;
    const int ncols = b.bc.P2 * b.KP();
    hipLaunchKernelGGL((k_zconv_b<L, SH>), dim3((ncols + NPB - 1) / NPB, 1, b.cap), dim3(NPB * TT), 0, b.st,
                       b.slots, b.tw);
}
template <int L>
void launch_zconv_bt(const BatchLaunch &b) {
    if constexpr (L <= 256) {
        switch (b.bc.tune_z) {
            case 1: if constexpr ((256 / fft2_threads(L)) >= 2) { launch_zconv_bsh<L, 1>(b); return; } break;
            case 2: if constexpr ((256 / fft2_threads(L)) >= 4) { launch_zconv_bsh<L, 2>(b); return; } break;
            default: break;
        }
        launch_zconv_bsh<L, 0>(b);
    }
}
template <int L>
void launch_yconv_bt(const BatchLaunch &b) {
    constexpr int TB = tb_triple(L);
    const int K1 = b.bc.P1 / 2 + 1;
    hipLaunchKernelGGL((k_yconv_b<L, TB>), dim3((K1 + TB - 1) / TB, 1, b.cap), dim3(yconv_threads(L)), 0, b.st,
                       b.slots, b.tw);
}
}  // namespace

hipError_t launch_batch_demag(const BatchClass &bc, const BatchSlot *slots, int cap, int stage, hipStream_t st) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const float2 *tw = twiddles(dev);
    if (!tw) return hipErrorOutOfMemory;
    if (bc.P3 > 256) return hipErrorInvalidValue;   // the register z convolution only
    const BatchLaunch b{bc, slots, cap, stage, st, tw};
    const int L1 = bc.P1 / 2;
    NM_DISPATCH_ROW(L1, launch_xfwd_bt, b);
    if (bc.P3 > 1) {
        NM_DISPATCH_COL(bc.P2, launch_yfwd_bt, b);
        NM_DISPATCH_COL(bc.P3, launch_zconv_bt, b);
        NM_DISPATCH_COL(bc.P2, launch_yinv_bt, b);
    } else {
        NM_DISPATCH_COL(bc.P2, launch_yconv_bt, b);
    }
    NM_DISPATCH_ROW(L1, launch_xinv_bt, b);
    return hipGetLastError();
}

hipError_t demag_forward_conv_inverse(nm_mesh *m, const float *mag, int src_mode) {
    return demag_pipeline(m, mag, nullptr, src_mode);
}

hipError_t demag_forward_conv_inverse_ctrl(nm_mesh *m, const float *mag, const Ctrl *ctrl,
                                           int src_mode) {
    return demag_pipeline(m, mag, ctrl, src_mode);
}

}  // namespace nm
