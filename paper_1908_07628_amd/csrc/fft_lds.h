// Batched 1-D complex FFTs staged through LDS (Stockham auto-sort, radix 8/4/2).
//
// A sequence of N elements lives in LDS at lds[base + i * es].  T = N / E threads
// cooperate on one sequence; each holds E elements per stage and performs E / R
// radix-R butterflies.  Stage s combines R sub-transforms of length Ns into one of
// length Ns * R:
//     v_r = x[j + r N / R] * w^(r (j mod Ns) N / (Ns R)),   v <- DFT_R(v),
//     y[(j - j mod Ns) R + j mod Ns + r Ns] = v_r,          j = 0 .. N/R - 1,
// which leaves the result in natural order.  DIR = -1 is the forward transform
// exp(-2 pi i n k / N), DIR = +1 the unnormalised inverse.  Twiddles come from a
// table tw[m] = exp(-2 pi i m / N) computed in double precision.
#pragma once

#include <hip/hip_runtime.h>

namespace eels {

// The fused form is written out, so every kernel that inlines it rounds the same way
// (left to contraction, the compiler may fuse either product depending on the code
// around it, and variants of one pass would then differ in the last bit).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// multiply by DIR * i
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2& a, float2& b) {
    float2 t = csub(a, b);
    a = cadd(a, b);
    b = t;
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    float2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = mul_i<DIR>(csub(v1, v3));
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
    if constexpr (R == 2) {
        dft2<DIR>(v[0], v[1]);
    } else if constexpr (R == 4) {
        dft4<DIR>(v[0], v[1], v[2], v[3]);
    } else {
        static_assert(R == 8, "radix");
        float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
        float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
        dft4<DIR>(e0, e1, e2, e3);
        dft4<DIR>(o0, o1, o2, o3);
        constexpr float h = 0.70710678118654752440f;
        // w = exp(DIR 2 pi i / 8): w^1 = h (1 + DIR i), w^2 = DIR i, w^3 = h (-1 + DIR i)
        float2 t1 = cmul(o1, make_float2(h, DIR * h));
        float2 t2 = mul_i<DIR>(o2);
        float2 t3 = cmul(o3, make_float2(-h, DIR * h));
        v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
        v[1] = cadd(e1, t1); v[5] = csub(e1, t1);
        v[2] = cadd(e2, t2); v[6] = csub(e2, t2);
        v[3] = cadd(e3, t3); v[7] = csub(e3, t3);
    }
}

template <int N, int Ns>
struct StageRadix {
    static constexpr int REM = N / Ns;
    static constexpr int R = REM >= 8 ? 8 : (REM >= 4 ? 4 : 2);
};

template <int N, int E, int DIR, int Ns>
__device__ __forceinline__ void fft_stages(float2* lds, int base, int es, int t, const float2* __restrict__ tw) {
    if constexpr (Ns < N) {
        constexpr int R = StageRadix<N, Ns>::R;
        constexpr int T = N / E;
        constexpr int NB = E / R;
        static_assert(NB * R == E && NB * T * R == N, "fft decomposition");
        float2 v[NB][R];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int j = t + b * T;
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = lds[base + (j + r * (N / R)) * es];
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            int j = t + b * T;
            int k = j & (Ns - 1);
            if constexpr (Ns > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    float2 w = tw[(r * k) * (N / (Ns * R))];
                    if (DIR > 0) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
            dft<R, DIR>(v[b]);
            int idxD = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) lds[base + (idxD + r * Ns) * es] = v[b][r];
        }
        __syncthreads();
        fft_stages<N, E, DIR, Ns * R>(lds, base, es, t, tw);
    }
}

// Full transform of one sequence per thread group; every thread of the block must call
// it (it contains barriers).
template <int N, int E, int DIR>
__device__ __forceinline__ void fft_lds(float2* lds, int base, int es, int t, const float2* __restrict__ tw) {
    fft_stages<N, E, DIR, 1>(lds, base, es, t, tw);
}

}  // namespace eels
