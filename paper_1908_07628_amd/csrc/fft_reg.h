// Register-resident Stockham FFT (radix 16 first, then 16/8/4/2; sides with a factor 3: radix
// 24 first, then 8 and 2), LDS only between stages.
//
// T = N / E threads cooperate on one sequence of length N; thread t holds the E elements
// t + T m (m = 0 .. E-1) in v[m], both on entry and on exit.  The first stage has radix
// E, so its butterfly j = t reads exactly v (inputs j + r N / E = t + r T); the last
// stage's outputs j + r N / R (j = t + b T) are again t + T (b + r E / R).  Middle
// stages exchange through lds[base + i * es] with a barrier on each side, so every
// thread of the block must call the transform the same number of times.
// PAD: element i sits at lds[base + (i + i / 16) * es].  A sequence's first exchange writes
// elements 16 t + r from thread t; unpadded, the lanes of neighbouring threads t (contiguous
// sequences, or interleaved ones es apart) meet in the same LDS banks, padded they spread over
// the banks.  The sequence then needs N + N / 16 slots (es apart).
// DIR = -1: forward exp(-2 pi i n k / N); DIR = +1: unnormalised inverse.
// WAVE: every sequence's T <= 64 threads lie in one wavefront (contiguous sequences of a
// row pass), so the exchanges need only wave-level ordering: a wavefront's LDS operations
// execute in program order, and the fences keep the compiler from moving LDS accesses
// across the exchange.  Otherwise block barriers separate the stages.
#pragma once

#include "fft_lds.h"

namespace eels {

__device__ __forceinline__ void lds_sync_wave() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int DIR>
__device__ __forceinline__ void dft16(float2* v) {
    // 16 = 4 x 4: x[4 n1 + n2] -> DFT4 over n1, twiddle W16^(n2 k1), DFT4 over n2
    float2 a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        float2 x0 = v[n2], x1 = v[4 + n2], x2 = v[8 + n2], x3 = v[12 + n2];
        dft4<DIR>(x0, x1, x2, x3);
        a[n2][0] = x0; a[n2][1] = x1; a[n2][2] = x2; a[n2][3] = x3;
    }
    constexpr float c1 = 0.92387953251128674f, s1 = 0.38268343236508978f, h = 0.70710678118654752f;
    // W16^p = exp(DIR 2 pi i p / 16), p = n2 k1 in {1, 2, 3, 2, 4, 6, 3, 6, 9}
    const float2 w1 = make_float2(c1, DIR * s1), w2 = make_float2(h, DIR * h), w3 = make_float2(s1, DIR * c1);
    const float2 w6 = make_float2(-h, DIR * h), w9 = make_float2(-c1, -DIR * s1);
    a[1][1] = cmul(a[1][1], w1); a[1][2] = cmul(a[1][2], w2); a[1][3] = cmul(a[1][3], w3);
    a[2][1] = cmul(a[2][1], w2); a[2][2] = mul_i<DIR>(a[2][2]); a[2][3] = cmul(a[2][3], w6);
    a[3][1] = cmul(a[3][1], w3); a[3][2] = cmul(a[3][2], w6); a[3][3] = cmul(a[3][3], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        float2 x0 = a[0][k1], x1 = a[1][k1], x2 = a[2][k1], x3 = a[3][k1];
        dft4<DIR>(x0, x1, x2, x3);
        v[k1] = x0; v[k1 + 4] = x1; v[k1 + 8] = x2; v[k1 + 12] = x3;
    }
}

// 3-point DFT: w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2
template <int DIR>
__device__ __forceinline__ void dft3(float2& a, float2& b, float2& c) {
    constexpr float h = 0.86602540378443865f;
    const float2 s = cadd(b, c), d = csub(b, c);
    const float2 m = make_float2(fmaf(-0.5f, s.x, a.x), fmaf(-0.5f, s.y, a.y));
    const float2 r = mul_i<DIR>(make_float2(h * d.x, h * d.y));
    a = cadd(a, s);
    b = cadd(m, r);
    c = csub(m, r);
}

template <int DIR>
__device__ __forceinline__ void dft24(float2* v) {
    // 24 = 3 x 8: x[8 n1 + n2] -> DFT3 over n1 (k1), twiddle W24^(n2 k1), DFT8 over n2 (k2);
    // X[k1 + 3 k2].  W24^p = cos(2 pi p / 24) + DIR i sin(2 pi p / 24), p = n2 k1 <= 14.
    constexpr float wc[15] = {1.0f, 0.9659258262890683f, 0.8660254037844387f, 0.7071067811865476f, 0.5000000000000001f, 0.25881904510252074f, 0.0f, -0.25881904510252063f, -0.4999999999999998f, -0.7071067811865475f, -0.8660254037844387f, -0.9659258262890682f, -1.0f, -0.9659258262890683f, -0.8660254037844388f};
    constexpr float ws[15] = {0.0f, 0.25881904510252074f, 0.49999999999999994f, 0.7071067811865475f, 0.8660254037844386f, 0.9659258262890683f, 1.0f, 0.9659258262890683f, 0.8660254037844387f, 0.7071067811865476f, 0.49999999999999994f, 0.258819045102521f, 0.0f, -0.2588190451025208f, -0.4999999999999997f};
    float2 a[3][8];
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) {
        float2 x0 = v[n2], x1 = v[8 + n2], x2 = v[16 + n2];
        dft3<DIR>(x0, x1, x2);
        a[0][n2] = x0;
        a[1][n2] = n2 == 0 ? x1 : cmul(x1, make_float2(wc[n2], DIR * ws[n2]));
        a[2][n2] = n2 == 0 ? x2 : cmul(x2, make_float2(wc[2 * n2], DIR * ws[2 * n2]));
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
        dft<8, DIR>(a[k1]);
#pragma unroll
        for (int k2 = 0; k2 < 8; ++k2) v[k1 + 3 * k2] = a[k1][k2];
    }
}

template <int R, int DIR>
__device__ __forceinline__ void dft_any(float2* v) {
    if constexpr (R == 16) dft16<DIR>(v);
    else if constexpr (R == 24) dft24<DIR>(v);
    else dft<R, DIR>(v);
}

// Elements per thread: 16 (radix-16 first stage) for powers of two; sides with a factor 3
// (384 = 3 x 128) hold 24 (a radix-24 = 3 x 8 first stage, then radices 8 and 2).
template <int N>
struct RegCfg {
    static constexpr int E = N % 3 == 0 ? 24 : (N >= 16 ? 16 : N);
    static constexpr int T = N / E;
};

// the largest radix of {16, 8, 4, 2} that divides both what is left of N and E
template <int N, int Ns, int E>
struct RegRadix {
    static constexpr int REM = N / Ns;
    static constexpr int R = (REM % 16 == 0 && E % 16 == 0) ? 16
                           : (REM % 8 == 0 && E % 8 == 0) ? 8 : (REM % 4 == 0 && E % 4 == 0) ? 4 : 2;
};

// stage with butterfly radix R on elements in registers (first stage) or LDS (later)
template <int N, int E, int DIR, int Ns, bool PAD, bool WAVE>
__device__ __forceinline__ void fft_reg_stages(float2 (&v)[E], float2* lds, int base, int es, int t,
                                               const float2* __restrict__ tw) {
    static_assert(!WAVE || N / E <= 64, "wave-local exchange needs the sequence in one wavefront");
    auto at = [&](int i) -> float2& { return PAD ? lds[base + (i + (i >> 4)) * es] : lds[base + i * es]; };
    constexpr int T = N / E;
    constexpr int R = (Ns == 1) ? E : RegRadix<N, Ns, E>::R;
    constexpr int NB = E / R;
    static_assert(NB * R == E && NB * T * R == N, "register fft decomposition");
    constexpr bool first = (Ns == 1);
    constexpr bool last = (Ns * R == N);
    float2 u[NB][R];
    if constexpr (first) {
#pragma unroll
        for (int r = 0; r < R; ++r) u[0][r] = v[r];
    } else {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int j = t + b * T;
#pragma unroll
            for (int r = 0; r < R; ++r) u[b][r] = at(j + r * (N / R));
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        int j = t + b * T;
        int k = (int)((unsigned)j % (unsigned)Ns);   // a mask for powers of two
        if constexpr (Ns > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                float2 w = tw[(r * k) * (N / (Ns * R))];
                if (DIR > 0) w.y = -w.y;
                u[b][r] = cmul(u[b][r], w);
            }
        }
        dft_any<R, DIR>(u[b]);
    }
    if constexpr (last) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < R; ++r) v[b + r * NB] = u[b][r];
    } else {
        // earlier readers of lds are done
        if constexpr (WAVE) lds_sync_wave();
        else __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int j = t + b * T;
            int k = (int)((unsigned)j % (unsigned)Ns);   // a mask for powers of two
            int idxD = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) at(idxD + r * Ns) = u[b][r];
        }
        if constexpr (WAVE) lds_sync_wave();
        else __syncthreads();
        fft_reg_stages<N, E, DIR, Ns * R, PAD, WAVE>(v, lds, base, es, t, tw);
    }
}

template <int N, int DIR, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_reg(float2 (&v)[RegCfg<N>::E], float2* lds, int base, int es, int t,
                                        const float2* __restrict__ tw) {
    fft_reg_stages<N, RegCfg<N>::E, DIR, 1, PAD, WAVE>(v, lds, base, es, t, tw);
}

// LDS slots of one padded contiguous sequence
template <int N>
struct PadLen {
    static constexpr int value = N + N / 16;
};

}  // namespace eels
