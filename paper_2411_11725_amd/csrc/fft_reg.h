// Register-resident FFTs for gfx950.
//
// dft_reg<R>: an R-point DFT (R <= 32) of values held in one thread's
// registers, natural order in and out; R > 8 splits as 4 x (R / 4) with
// compile-time twiddles.
//
// fft2: a length-L transform of a pencil spread over T = min(L1, L2) threads
// (L = L1 L2, four-step form): each thread does its L2-point DFTs, applies the
// twiddles W_L^(n1 k2), the block trades values once through LDS, and each
// thread does its L1-point DFTs.  Every element passes through LDS once per
// transform (one write, one read), where a radix-8 Stockham sweep in LDS
// reads and writes every element in every pass.
#pragma once

#include "fft_engine.h"

namespace nm {

// cos and sin of 2 pi q / 32
__host__ __device__ constexpr float cos32(int q) {
    constexpr float t[32] = {
        1.000000000e+00f,  9.807852804e-01f,  9.238795325e-01f,  8.314696123e-01f,
        7.071067812e-01f,  5.555702330e-01f,  3.826834324e-01f,  1.950903220e-01f,
        0.0f,             -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
        -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f,
        -1.000000000e+00f, -9.807852804e-01f, -9.238795325e-01f, -8.314696123e-01f,
        -7.071067812e-01f, -5.555702330e-01f, -3.826834324e-01f, -1.950903220e-01f,
        0.0f,              1.950903220e-01f,  3.826834324e-01f,  5.555702330e-01f,
        7.071067812e-01f,  8.314696123e-01f,  9.238795325e-01f,  9.807852804e-01f};
    return t[q & 31];
}
__host__ __device__ constexpr float sin32(int q) { return cos32(q - 8); }

// v * exp(DIR 2 pi i m / R); m is a compile-time constant after unrolling
template <int R, int DIR>
__device__ __forceinline__ float2 rot(float2 v, int m) {
    static_assert(32 % R == 0, "R divides 32");
    const int q = (m % R) * (32 / R);
    if (q == 0) return v;
    if (q == 8) return mul_dir_i<DIR>(v);            // DIR i
    if (q == 16) return make_float2(-v.x, -v.y);
    if (q == 24) return mul_dir_i<-DIR>(v);          // -DIR i
    const float c = cos32(q), s = DIR < 0 ? -sin32(q) : sin32(q);
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
}

// X_k = sum_n x_n exp(DIR 2 pi i n k / R), in place, natural order.
// ZH: the inputs x_n, n >= R/2, are zero (not read); OH: only X_k, k < R/2,
// are wanted (the upper outputs are left unspecified).  Zero padding makes
// half of every forward input and inverse output of the demag transforms
// such, and skipping them saves a butterfly stage's work.
template <int R, int DIR, bool ZH = false, bool OH = false>
__device__ __forceinline__ void dft_reg(float2 *v) {
    if constexpr (R <= 8) {
        if constexpr (R > 1) dft_small<R, DIR, ZH, OH>(v);
    } else {
        static_assert(R == 16 || R == 32, "R <= 32");
        constexpr int A = 4, B = R / 4;
        float2 t[R];
#pragma unroll
        for (int n1 = 0; n1 < A; ++n1) {
            // x_{n1 + A n2} with n2 >= B / 2 lies in the upper half
            float2 u[B];
#pragma unroll
            for (int n2 = 0; n2 < B; ++n2) u[n2] = (ZH && n2 >= B / 2) ? make_float2(0.f, 0.f) : v[n1 + A * n2];
            dft_reg<B, DIR, ZH>(u);
#pragma unroll
            for (int k2 = 0; k2 < B; ++k2) t[n1 * B + k2] = rot<R, DIR>(u[k2], n1 * k2);
        }
#pragma unroll
        for (int k2 = 0; k2 < B; ++k2) {
            // X_{k2 + B k1} with k1 >= A / 2 lies in the upper half
            float2 u[A];
#pragma unroll
            for (int n1 = 0; n1 < A; ++n1) u[n1] = t[n1 * B + k2];
            dft_small<A, DIR, false, OH>(u);
#pragma unroll
            for (int k1 = 0; k1 < (OH ? A / 2 : A); ++k1) v[k2 + B * k1] = u[k1];
        }
    }
}

// split of a length-L pencil: L1 x L2, threads per pencil T, values per thread E
__host__ __device__ constexpr int fft2_l1(int L) {
    return L <= 8 ? 1 : L == 16 ? 4 : L <= 64 ? 8 : L <= 256 ? 16 : 32;
}
__host__ __device__ constexpr int fft2_threads(int L) {
    return fft2_l1(L) < L / fft2_l1(L) ? fft2_l1(L) : L / fft2_l1(L);
}
inline int fft2_threads_host(int L) { return fft2_threads(L); }

// LDS copy tl[j] = exp(-2 pi i j / L), j < L (full period)
template <int L, int NT>
__device__ __forceinline__ void load_twiddles_full(float2 *tl, const float2 *__restrict__ tw, int tid) {
    static_assert(L <= kTwN && kTwN % L == 0, "table period");
    for (int q = tid; q < L; q += NT) tl[q] = tw[q * (kTwN / L)];
}

// NC components of one pencil per thread group, length L = L1 L2 each,
// T = min(L1, L2) threads per pencil (j = 0 .. T-1), NPB pencils per block
// (b = 0 .. NPB-1), E = L / T values per thread and component:
//   in   v[c][a * L2 + n2] = x_c[(j + T a) + L1 n2],   a < L1 / T, n2 < L2
//   out  v[c][q * L1 + k1] = X_c[(j + T q) + L2 k1],   q < L2 / T, k1 < L1
// The inverse of a forward (L1, L2) transform is fft2<L2, L1, +1>: it takes
// the forward output layout as input and returns the forward input layout.
// sh holds NC L NPB complex values (element e of pencil b, component c at
// sh[(c L + e) NPB + b]: consecutive lanes, consecutive pencils); tl is a
// forward twiddle table of period L.  Begins with a block barrier (sh and tl
// must be free / ready), so every thread of the block must call it.
//
// ZIN: the inputs with n2 >= L2 / 2 (the upper half of x) are zero; ZOUT:
// only the outputs with k1 < L1 / 2 (the lower half of X) are wanted.
template <int L1, int L2, int DIR, int NC, int NPB, int E, bool ZIN = false, bool ZOUT = false>
__device__ __forceinline__ void fft2(float2 (&v)[NC][E], float2 *sh, const float2 *tl, int j, int b) {
    constexpr int L = L1 * L2;
    constexpr int T = L1 < L2 ? L1 : L2;
    static_assert(E == L / T, "values per thread");
    if constexpr (T == 1) {
#pragma unroll
        for (int c = 0; c < NC; ++c) dft_reg<L, DIR, ZIN, ZOUT>(v[c]);
    } else {
        constexpr int A = L1 / T, Q = L2 / T;
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int a = 0; a < A; ++a) dft_reg<L2, DIR, ZIN>(&v[c][a * L2]);
        __syncthreads();
#pragma unroll
        for (int a = 0; a < A; ++a) {
            const int n1 = j + T * a;
#pragma unroll
            for (int k2 = 0; k2 < L2; ++k2) {
                float2 w = make_float2(1.f, 0.f);
                if (k2 > 0) w = twiddle<DIR>(tl, n1 * k2);   // n1 k2 < L
#pragma unroll
                for (int c = 0; c < NC; ++c)
                    sh[(c * L + k2 * L1 + n1) * NPB + b] = k2 == 0 ? v[c][a * L2] : cmul(v[c][a * L2 + k2], w);
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q)
#pragma unroll
                for (int n1 = 0; n1 < L1; ++n1) v[c][q * L1 + n1] = sh[(c * L + (j + T * q) * L1 + n1) * NPB + b];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < Q; ++q) dft_reg<L1, DIR, false, ZOUT>(&v[c][q * L1]);
    }
}

}  // namespace nm
