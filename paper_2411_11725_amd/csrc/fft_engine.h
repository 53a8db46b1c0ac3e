// In-LDS batched complex FFT for power-of-two lengths 2..1024 (gfx950).
//
// A workgroup transforms NP pencils of length L held in LDS.  Each pass is a
// Stockham auto-sort step of radix 8, 4 or 2: a thread loads the R inputs of
// one butterfly into registers, applies the twiddles w^(r k) (from a float64-
// built table), does the radix-R DFT in registers and writes the outputs in
// natural order for the next pass.  Two layouts:
//   element-major (EM = true):  element i of pencil p at s[i * NP + p]
//     (column tiles of the y / z passes; consecutive lanes = consecutive
//     pencils, so LDS accesses never conflict)
//   pencil-major  (EM = false): s[p * L + i]   (rows of the x pass)
#pragma once

#include <hip/hip_runtime.h>

#include "nm_internal.h"

namespace nm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// multiply by DIR * i  (DIR = -1 forward, +1 inverse)
template <int DIR>
__device__ __forceinline__ float2 mul_dir_i(float2 v) {
    return DIR < 0 ? make_float2(v.y, -v.x) : make_float2(-v.y, v.x);
}

// exp(DIR * 2 pi i t / N) from a forward table of period N (the global table
// has N = kTwN; kernels copy the entries they need into LDS with a shorter
// period, see load_twiddles)
template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2 *__restrict__ tw, int t) {
    float2 w = tw[t];
    return DIR < 0 ? w : make_float2(w.x, -w.y);
}

// LDS copy tl[j] = exp(-2 pi i j / TWL), j = 0 .. TWL/2, of the global table.
// Call after the kernel's data loads are issued: the copy's one memory round
// trip then overlaps theirs, and every FFT pass reads its twiddles from LDS.
template <int TWL, int NT>
__device__ __forceinline__ void load_twiddles(float2 *tl, const float2 *__restrict__ tw, int tid) {
    static_assert(TWL >= 2 && TWL <= kTwN && kTwN % TWL == 0, "table period");
    for (int j = tid; j <= TWL / 2; j += NT) tl[j] = tw[j * (kTwN / TWL)];
}

template <int R, int DIR, bool ZH = false, bool OH = false>
__device__ __forceinline__ void dft_small(float2 *v) {
    // ZH: inputs v[R/2 ..] are zero (and are not read); OH: only the outputs
    // v[0 .. R/2) are wanted (the others are left as they are)
    if constexpr (R == 2) {
        if constexpr (ZH) {
            v[1] = v[0];
        } else {
            float2 a = v[0], b = v[1];
            v[0] = cadd(a, b);
            if constexpr (!OH) v[1] = csub(a, b);
        }
    } else if constexpr (R == 4) {
        if constexpr (ZH) {
            const float2 a = v[0], b = v[1], d = mul_dir_i<DIR>(v[1]);
            v[0] = cadd(a, b);
            v[1] = cadd(a, d);
            if constexpr (!OH) {
                v[2] = csub(a, b);
                v[3] = csub(a, d);
            }
        } else {
            float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
            float2 s13 = cadd(v[1], v[3]), d13 = mul_dir_i<DIR>(csub(v[1], v[3]));
            v[0] = cadd(s02, s13);
            v[1] = cadd(d02, d13);
            if constexpr (!OH) {
                v[2] = csub(s02, s13);
                v[3] = csub(d02, d13);
            }
        }
    } else {  // R == 8: two radix-4 halves joined by w8^k
        float2 e[4] = {v[0], v[2], make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        float2 o[4] = {v[1], v[3], make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
        if constexpr (!ZH) {
            e[2] = v[4];
            e[3] = v[6];
            o[2] = v[5];
            o[3] = v[7];
        }
        dft_small<4, DIR, ZH>(e);
        dft_small<4, DIR, ZH>(o);
        const float r = 0.70710678118654752440f;
        // w8^1 = (1 + DIR i)/sqrt2, w8^2 = DIR i, w8^3 = (-1 + DIR i)/sqrt2
        float2 o1 = cscale(cadd(o[1], mul_dir_i<DIR>(o[1])), r);
        float2 o2 = mul_dir_i<DIR>(o[2]);
        float2 o3 = cscale(csub(mul_dir_i<DIR>(o[3]), o[3]), r);
        v[0] = cadd(e[0], o[0]);
        v[1] = cadd(e[1], o1);
        v[2] = cadd(e[2], o2);
        v[3] = cadd(e[3], o3);
        if constexpr (!OH) {
            v[4] = csub(e[0], o[0]);
            v[5] = csub(e[1], o1);
            v[6] = csub(e[2], o2);
            v[7] = csub(e[3], o3);
        }
    }
}

// radix of the next pass for a remaining length 2^m: 8s, with a 4 (or two)
// instead of a trailing 2
__host__ __device__ constexpr int radix_for(int rem) {
    return rem == 2 ? 2 : rem == 4 ? 4 : rem == 16 ? 4
         : (rem == 8 || rem == 64 || rem == 512 || rem == 4096) ? 8
         : (rem == 128 || rem == 1024) ? 4 : 8;
}

template <int L, int NP, bool EM>
__device__ __forceinline__ int lds_index(int p, int i) {
    return EM ? i * NP + p : p * L + i;
}

template <int L, int R, int NS, int DIR, int NP, int NT, bool EM, int TWL>
__device__ __forceinline__ void fft_pass(float2 *s, const float2 *__restrict__ tw, int tid) {
    constexpr int J = L / R;
    constexpr int JOBS = NP * J;
    constexpr int JPT = (JOBS + NT - 1) / NT;
    float2 v[JPT][R];
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
        const int job = tid + q * NT;
        if (JOBS % NT == 0 || job < JOBS) {
            const int p = EM ? job % NP : job / J;
            const int j = EM ? job / NP : job % J;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = s[lds_index<L, NP, EM>(p, j + r * J)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JPT; ++q) {
        const int job = tid + q * NT;
        if (JOBS % NT == 0 || job < JOBS) {
            const int p = EM ? job % NP : job / J;
            const int j = EM ? job / NP : job % J;
            const int k = j % NS;
            if constexpr (NS > 1) {
                // w^r, r < R, from the table entries w, w^2, w^4 (one extra
                // rounding at most for the products); 4 k stride < TWL / 2
                static_assert(TWL % (NS * R) == 0, "table period");
                constexpr int stride = TWL / (NS * R);
                const float2 w1 = twiddle<DIR>(tw, k * stride);
                if constexpr (R == 2) {
                    v[q][1] = cmul(v[q][1], w1);
                } else {
                    const float2 w2 = twiddle<DIR>(tw, 2 * k * stride);
                    const float2 w3 = cmul(w1, w2);
                    v[q][1] = cmul(v[q][1], w1);
                    v[q][2] = cmul(v[q][2], w2);
                    v[q][3] = cmul(v[q][3], w3);
                    if constexpr (R == 8) {
                        const float2 w4 = twiddle<DIR>(tw, 4 * k * stride);
                        v[q][4] = cmul(v[q][4], w4);
                        v[q][5] = cmul(v[q][5], cmul(w1, w4));
                        v[q][6] = cmul(v[q][6], cmul(w2, w4));
                        v[q][7] = cmul(v[q][7], cmul(w3, w4));
                    }
                }
            }
            dft_small<R, DIR>(v[q]);
            const int base = (j / NS) * NS * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) s[lds_index<L, NP, EM>(p, base + r * NS)] = v[q][r];
        }
    }
    __syncthreads();
}

template <int L, int NS, int DIR, int NP, int NT, bool EM, int TWL>
__device__ __forceinline__ void fft_passes(float2 *s, const float2 *__restrict__ tw, int tid) {
    if constexpr (NS < L) {
        constexpr int R = radix_for(L / NS);
        fft_pass<L, R, NS, DIR, NP, NT, EM, TWL>(s, tw, tid);
        fft_passes<L, NS * R, DIR, NP, NT, EM, TWL>(s, tw, tid);
    }
}

// Unnormalised DFT of NP pencils in LDS: X_k = sum_n x_n exp(DIR 2 pi i n k / L).
// tw is a forward twiddle table of period TWL (a multiple of L), e.g. the LDS
// copy from load_twiddles.  Expects the data written and a barrier passed;
// ends with a barrier.
template <int L, int DIR, int NP, int NT, bool EM, int TWL>
__device__ __forceinline__ void lds_fft(float2 *s, const float2 *__restrict__ tw, int tid) {
    static_assert(TWL % L == 0, "table period");
    fft_passes<L, 1, DIR, NP, NT, EM, TWL>(s, tw, tid);
}

}  // namespace nm
