// Multislice sweeps of the scattering matrices and the small set-up kernels.
//
// A beam's wave is kept between slices in the hybrid (kx, y) representation, stored
// as [beam][y][ldx] over the nlx kx columns inside the band limit (see phys_col_of).
// One slice of the forward operator M_j = P_j F T_j F^-1 (Eq. MSop) is two passes over HBM:
//   row pass     iFFT_x -> (capture S_1 windows) -> * T_j -> FFT_x
//   column pass  FFT_y  -> * P_j / (nx ny)       -> iFFT_y
// one slice of the exact transpose M_j^T = F^-1 T_j F P_j used for S_2 is
//   column pass  iFFT_y -> * P_j / (nx ny)       -> FFT_y
//   row pass     FFT_x  -> * T_j -> (capture S_2 windows) -> iFFT_x
// and one slice of the inverse multislice M_j^-1 = F conj(T_j) F^-1 conj(P_j) (Eq. MSinvop),
// which retreats S_1 by a slice, is
//   column pass  FFT_y  -> * conj(P_j) / (nx ny) -> iFFT_y
//   row pass     iFFT_x -> * conj(T_j) -> (capture S_1 windows) -> FFT_x
// while the inverse of a transposed step, (M_j^T)^-1 = conj(P_j) F^-1 conj(T_j) F, which
// retreats S_2 by a slice towards the exit (mode 3), is
//   row pass     FFT_x  -> (capture S_2 windows) -> * conj(T_j) -> iFFT_x
//   column pass  iFFT_y -> * conj(P_j) / (nx ny) -> FFT_y
// The retreat starts from the transposed sweep's state before the row pass of slice 0, which is
// still band-limited; its first row pass (mode 4) is
//   row pass     FFT_x  -> * T_j -> (capture S_2 windows) -> * conj(T_j) nx -> iFFT_x
// which captures what the transposed sweep captures there and stores its input times nx^2.
// Transforms are unnormalised; the 1/(nx ny) folded into P keeps S_2 exactly at the
// scale of its definition and S_1 at nx*ny times it (unit-modulus plane waves at j = 0).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fft_lds.h"
#include "fft_reg.h"
#include "internal.h"
#include "kernels.h"
#include "stream_store.h"

namespace eels {

// Split-complex store (see the GEMM kernels): slot `off` of an SC array.
__device__ __forceinline__ uint32_t bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ void split_c(float2 v, int sc, uint32_t& hi, uint32_t& lo) {
    if (sc == EELS_BF16_SPLIT) {
        uint32_t ha = bf16_rne(v.x), hb = bf16_rne(v.y);
        float ra = v.x - __uint_as_float(ha << 16), rb = v.y - __uint_as_float(hb << 16);
        hi = ha | (hb << 16);
        lo = bf16_rne(ra) | (bf16_rne(rb) << 16);
    } else {
        _Float16 ha = (_Float16)v.x, hb = (_Float16)v.y;
        _Float16 la = (_Float16)(v.x - (float)ha), lb = (_Float16)(v.y - (float)hb);
        hi = (uint32_t)__builtin_bit_cast(uint16_t, ha) | ((uint32_t)__builtin_bit_cast(uint16_t, hb) << 16);
        lo = (uint32_t)__builtin_bit_cast(uint16_t, la) | ((uint32_t)__builtin_bit_cast(uint16_t, lb) << 16);
    }
}
__device__ __forceinline__ void store_c(void* base, int64_t off, float2 v, int sc) {
    if (sc == 0) {
        st_stream((float2*)base + off, v);
        return;
    }
    uint32_t hi, lo;
    split_c(v, sc, hi, lo);
    uint32_t* b = (uint32_t*)base;
    int64_t u = off >> 2;
    int pos = (int)(off & 3);
    st_stream(b + u * 8 + pos, hi);
    st_stream(b + u * 8 + 4 + pos, lo);
}

// --------------------------------------------------------------------- set-up kernels

__global__ void k_twiddles(float2* tw, int n) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    double s, c;
    sincospi(-2.0 * (double)m / (double)n, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
}

// T_j(r) = exp(i sigma V_j(r))
__global__ void k_transmission(float2* T, const float* V, int64_t n, double sigma) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s, c;
    sincos(sigma * (double)V[i], &s, &c);
    T[i] = make_float2((float)c, (float)s);
}

__device__ __forceinline__ int signed_index(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

__device__ __forceinline__ int live_to_kx_signed(int c, int nlx, int hlx, int nx) {
    if (nlx == nx) return signed_index(c, nx);
    return c <= hlx ? c : c - nlx;
}

// P~_j(kx, ky) = B(k) exp(-i pi lambda dz_j |k|^2) / (nx ny) on the live columns; the band
// B is |ky index| <= band_h[c] for live column c (the host's table, shared with the band
// captures so that every kernel agrees on the band pixel set)
// Separable propagator of slice j (Eq. MSop with the band limit): P_j(kx, ky) = px_j[c] py_j[y]
// inside the band (|signed y| <= band_h[c]), 0 outside, with px_j[c] = exp(-i pi lam dz kx^2) /
// (nx ny) on the live columns and py_j[y] = exp(-i pi lam dz ky^2).  Slice j's tables sit at
// P + j (nlx + ny): nlx column factors, then ny row factors (phases in double).
__global__ void k_propagator(float2* P, const double* dz, int nz, int nx, int ny, int nlx, int hlx, double lx,
                             double ly, double lam) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int per = nlx + ny;
    if (i >= (int64_t)nz * per) return;
    const int j = (int)(i / per), r = (int)(i % per);
    double k, sc;
    if (r < nlx) {
        k = live_to_kx_signed(r, nlx, hlx, nx) / lx;
        sc = 1.0 / ((double)nx * (double)ny);
    } else {
        k = signed_index(r - nlx, ny) / ly;
        sc = 1.0;
    }
    double s, co;
    sincospi(-lam * dz[j] * k * k, &s, &co);
    P[i] = make_float2((float)(co * sc), (float)(s * sc));
}

// c_k(R) = s exp(-i chi(k)) exp(-2 pi i k.R), stored [P][N1pad] (zero padding columns).
// The scan phase is reduced to a fraction of a cycle in double before the sincos.
__global__ void k_probe_coefficients(void* C, const int4* beams, int N1, int N1pad, const double* probes, int P,
                                     int f, double lx, double ly, double lam, double defocus, double cs,
                                     double scale, int sc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P * N1pad) return;
    int k = (int)(i % N1pad);
    int r = (int)(i / N1pad);
    float2 out = make_float2(0.f, 0.f);
    if (k < N1) {
        int4 b = beams[k];
        double kx = (double)(f * b.z) / lx, ky = (double)(f * b.w) / ly;
        double u = kx * probes[2 * r] + ky * probes[2 * r + 1];
        u -= floor(u);
        double k2 = kx * kx + ky * ky;
        double chi = M_PI * lam * k2 * (0.5 * cs * lam * lam * k2 - defocus);
        double s, c;
        sincos(-2.0 * M_PI * u - chi, &s, &c);
        out = make_float2((float)(c * scale), (float)(s * scale));
    }
    store_c(C, i, out, sc);
}

// Live kx columns are stored in rows of ldx (nlx rounded up to 16) complex: |kx| <= hlx
// at x for x <= hlx and at x - N + ldx for x >= N - hlx (right-aligned), so a physical
// column is congruent to its pixel x modulo 16 and 16-column segments are 128-byte aligned.
// Returns -1 for the dead columns.  (Without pruning, nlx = ldx = N and this is x.)
__device__ __forceinline__ int phys_col_of(int x, int N, int hlx, int ldx) {
    return x <= hlx ? x : (x >= N - hlx ? x - N + ldx : -1);
}
// physical column -> logical live column index (0 .. nlx-1), -1 in the gap or beyond ldx
// (nlx == ldx only without pruning, where both maps are the identity; otherwise nlx is odd
// and hlx = (nlx - 1) / 2)
__device__ __forceinline__ int logical_of_phys(int pc, int nlx, int ldx) {
    if (pc >= ldx) return -1;
    if (nlx == ldx) return pc;
    const int hlx = (nlx - 1) / 2;
    return pc <= hlx ? pc : (pc >= ldx - hlx ? pc - (ldx - nlx) : -1);
}
__device__ __forceinline__ int phys_of_logical(int c, int nlx, int ldx) {
    if (nlx == ldx) return c;
    return c <= (nlx - 1) / 2 ? c : c + (ldx - nlx);
}

// Forward sweep start: beam b = plane wave e_k, in (kx, y): column col_b holds exp(2 pi i ky y / ny).
__global__ void k_init_forward(float2* S, const int4* beams, int nb, int ny, int nlx, int ldx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * ny * nlx;
    if (i >= total) return;
    int c = (int)(i % nlx);
    int y = (int)((i / nlx) % ny);
    int b = (int)(i / ((int64_t)nlx * ny));
    int4 bm = beams[b];
    float2 out = make_float2(0.f, 0.f);
    if (c == bm.x) {
        int m = (int)(((int64_t)bm.y * y) % ny);
        double s, co;
        sincospi(2.0 * (double)m / (double)ny, &s, &co);
        out = make_float2((float)co, (float)s);
    }
    S[((int64_t)b * ny + y) * ldx + phys_of_logical(c, nlx, ldx)] = out;
}

// Reverse sweep start: w = fft_y(P_{nz-1} e_q): column col_q holds P(q) exp(-2 pi i qy y / ny).
__global__ void k_init_reverse(float2* S, const int4* beams, int nb, int ny, int nlx, int ldx, int f, double lx, double ly,
                               double lam, double dz_last) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nb * ny * nlx;
    if (i >= total) return;
    int c = (int)(i % nlx);
    int y = (int)((i / nlx) % ny);
    int b = (int)(i / ((int64_t)nlx * ny));
    int4 bm = beams[b];
    float2 out = make_float2(0.f, 0.f);
    if (c == bm.x) {
        double kx = (double)(f * bm.z) / lx, ky = (double)(f * bm.w) / ly;
        int m = (int)(((int64_t)bm.y * y) % ny);
        double ph = -lam * dz_last * (kx * kx + ky * ky) - 2.0 * (double)m / (double)ny;  // in units of pi
        double s, co;
        sincospi(ph, &s, &co);
        out = make_float2((float)co, (float)s);
    }
    S[((int64_t)b * ny + y) * ldx + phys_of_logical(c, nlx, ldx)] = out;
}

__global__ void k_fill_zero(float4* p, int64_t n4) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n4; i += stride) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void k_fill_zero_d(double* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// Copy real-space rows of a window buffer holding full planes (diagnostics).
__global__ void k_copy(float2* dst, const float2* src, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// --------------------------------------------------------------------- row pass
//
// T = N/16 threads per row, 16 elements each (pixel / column t + T m in v[m]); a group of
// S = 256/T rows of the flat row index g = beam * ny + y per block iteration.  Loads and
// stores go straight between HBM and registers; only the middle FFT stages use LDS.  A
// block walks the row groups blockIdx.x, blockIdx.x + gridDim.x, ... and loads the next
// group's rows into registers while it transforms the current one, so HBM traffic
// overlaps the FFT arithmetic of the same wave (the grid is capped, see row_grid).
// mode 0: forward sweep (iFFT_x, capture, x T, FFT_x); mode 1: transposed sweep (FFT_x, x T,
// capture, iFFT_x); mode 2: inverse multislice, Eq. MSinvop (iFFT_x, x conj(T), capture the
// slice's entrance wave, FFT_x); mode 3: the transposed step undone (FFT_x, capture the S_2 row
// of this slice, x conj(T), iFFT_x).  CAP = false: no capture (its code and registers left out).
template <int N, int MODE, bool CAP>
__device__ __forceinline__ void row_pass_body(float2* __restrict__ state, int nbeam, int ny, int nlx, int hlx, int ldx,
                                              const float2* __restrict__ Tj, const float2* __restrict__ tw,
                                              const int* __restrict__ cap_ptr, const int4* __restrict__ cap_rec,
                                              void* __restrict__ win, int64_t win_beams, int Kpad, int sc,
                                              float2* lds, const float2* __restrict__ cfac = nullptr) {
    constexpr int E = RegCfg<N>::E, T = RegCfg<N>::T, S = 256 / T, L = PadLen<N>::value;
    const int tid = threadIdx.x, s = tid / T, t = tid % T;
    const int64_t total = (int64_t)nbeam * ny;
    const int64_t ngroups = (total + S - 1) / S;
    float2 nxt[E];
    auto load = [&](int64_t grp) {
        const int64_t g = grp * S + s;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            int c = phys_col_of(t + T * m, N, hlx, ldx);
            nxt[m] = (g < total && c >= 0) ? state[g * ldx + c] : make_float2(0.f, 0.f);
        }
    };
    if ((int64_t)blockIdx.x < ngroups) load(blockIdx.x);
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        float2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = nxt[m];
        const int64_t g = grp * S + s;
        const bool valid = g < total;
        const int y = valid ? (int)(g % ny) : 0;
        const int64_t beam = valid ? g / ny : 0;
        if (grp + gridDim.x < ngroups) load(grp + gridDim.x);
        constexpr int S1 = (MODE == 1 || MODE >= 3) ? -1 : +1;   // first transform's sign (+1: inverse FFT_x)
        fft_reg<N, S1, true, true>(v, lds, s * L, 1, t, tw);

        // In mode 2 the column pass's conj(P_j) / (nx ny) leaves this pass's input 1/nx of the
        // forward row pass's output (the state after the final FFT_x is exact), so the captured
        // entrance wave is scaled by nx (exact) to match the forward capture.
        // In mode 3 the row's FFT_x of the transposed sweep's state is N times the S_2 row that
        // the transposed sweep captured at this slice (its FFT_x / iFFT_x pair is unnormalised),
        // so the capture is scaled by 1/N (exact).
        constexpr float cap_scale = MODE == 2 ? (float)N : MODE == 3 ? 1.0f / (float)N : 1.0f;
        // Capture: the row is put in pixel order into its own exchange slots (free between the
        // two transforms; a row's T <= 64 threads are one wave, whose LDS operations complete
        // in order), then the window rows it meets are written as one flat run of
        // (record, pixel) pairs, T pairs per store, so that each store covers whole window rows
        // back to back instead of one partly filled store per record.
        auto capture = [&]() {
            if constexpr (CAP) {
                float2* crow = lds + s * L;
                lds_sync_wave();
                if (cfac) {
                    // the beam's factor (times the capture scale) goes into every captured value
                    const float2 cb = cfac[beam];
                    const float2 cs = make_float2(cb.x * cap_scale, cb.y * cap_scale);
#pragma unroll
                    for (int m = 0; m < E; ++m) crow[t + T * m] = cmul(v[m], cs);
                } else {
#pragma unroll
                    for (int m = 0; m < E; ++m) crow[t + T * m] = make_float2(v[m].x * cap_scale, v[m].y * cap_scale);
                }
                lds_sync_wave();
                if (valid) {
                    // the row's records are fetched T at a time, one per thread; a pair's record
                    // comes from its owner by a shuffle.  Every record of a plan has the same
                    // width nw (the window's, or the whole row), so pair f belongs to record
                    // f / nw, found exactly in FP32 (f < 64 nw, nw <= 1024).  The trip count is
                    // the same for the row's T threads, so the shuffles always read active lanes.
                    const int r0 = cap_ptr[y], cnt = cap_ptr[y + 1] - r0;
                    const int64_t bbase = beam * (int64_t)Kpad;
                    for (int c0 = 0; c0 < cnt; c0 += T) {
                        const int4 mine = c0 + t < cnt ? cap_rec[r0 + c0 + t] : make_int4(0, 0, 0, 0);
                        const int n = min(T, cnt - c0);
                        const int nw = __shfl(mine.w, 0, T);
                        const int pk = mine.z * 2048 + mine.y;    // x0 and dy (both < 2048)
                        const float inv = 1.0f / (float)nw;
                        const int tot = n * nw, iters = (tot + T - 1) / T;
#pragma unroll 4
                        for (int k = 0; k < iters; ++k) {
                            const int f = min(t + T * k, tot - 1);
                            const int i = (int)(((float)f + 0.5f) * inv);
                            const int u = f - i * nw;
                            const int win_i = __shfl(mine.x, i, T), xy = __shfl(pk, i, T);
                            int px = (xy >> 11) + u;
                            if (px >= N) px -= N;
                            const int64_t dst = (int64_t)win_i * win_beams * Kpad + bbase + (int64_t)(xy & 2047) * nw + u;
                            if (t + T * k < tot) store_c(win, dst, crow[px], sc);
                        }
                    }
                }
                lds_sync_wave();
            }
        };
        if constexpr (MODE == 0 || MODE == 3) capture();
        const float2* Trow = Tj + (int64_t)y * N;
#pragma unroll
        for (int m = 0; m < E; ++m) {
            float2 tv = Trow[t + T * m];
            if constexpr (MODE == 2 || MODE == 3) tv.y = -tv.y;
            v[m] = cmul(v[m], tv);
        }
        if constexpr (MODE == 1 || MODE == 2 || MODE == 4) capture();
        if constexpr (MODE == 4) {
            // the row's T_j goes to the capture only: undo it, with the factor N that makes the
            // stored row N^2 times its input (the scale the retreat's column pass expects)
#pragma unroll
            for (int m = 0; m < E; ++m) {
                float2 tv = Trow[t + T * m];
                tv.x *= (float)N;
                tv.y *= -(float)N;
                v[m] = cmul(v[m], tv);
            }
        }

        fft_reg<N, -S1, true, true>(v, lds, s * L, 1, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            int c = phys_col_of(t + T * m, N, hlx, ldx);
            if (valid && c >= 0) state[g * ldx + c] = v[m];
        }
    }
}

// Two waves per SIMD, with and without capture (at N = 1024 the capturing variant spills
// 36 bytes per lane to get there, and is faster for it than at one wave); one wave for the
// 24-element sequences of the sides with a factor 3, whose registers do not fit two.
template <int N, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RegCfg<N>::E > 16 ? 1 : 2))) void k_row_pass(
    float2* __restrict__ state, int nbeam, int ny, int nlx, int hlx, int ldx, const float2* __restrict__ Tj,
    const float2* __restrict__ tw) {
    __shared__ float2 lds[(256 / RegCfg<N>::T) * PadLen<N>::value];
    row_pass_body<N, MODE, false>(state, nbeam, ny, nlx, hlx, ldx, Tj, tw, nullptr, nullptr, nullptr, 0, 0, 0, lds);
}

template <int N, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RegCfg<N>::E > 16 ? 1 : 2))) void k_row_pass_cap(float2* __restrict__ state, int nbeam, int ny, int nlx, int hlx,
                                                      int ldx, const float2* __restrict__ Tj,
                                                      const float2* __restrict__ tw, const int* __restrict__ cap_ptr,
                                                      const int4* __restrict__ cap_rec, void* __restrict__ win,
                                                      int64_t win_beams, int Kpad, int sc,
                                                      const float2* __restrict__ cfac) {
    __shared__ float2 lds[(256 / RegCfg<N>::T) * PadLen<N>::value];
    row_pass_body<N, MODE, true>(state, nbeam, ny, nlx, hlx, ldx, Tj, tw, cap_ptr, cap_rec, win, win_beams, Kpad, sc,
                                 lds, cfac);
}

// --------------------------------------------------------------------- column pass
//
// A block transforms CW live columns of one beam along y: thread (col, t), col = tid % CW,
// holds rows t + T m of its column in registers (rows of the strip are CW * 8 bytes
// contiguous in HBM).
template <int N>
struct ColCfg {
    static constexpr int T = RegCfg<N>::T;
    static constexpr int E = RegCfg<N>::E;
    static constexpr int NT = N >= 512 ? 512 : 256;
    static constexpr int CW = NT / T;
};

template <int N, int MODE, bool CAP>
__device__ __forceinline__ void col_pass_body(float2* __restrict__ state, int nbeam, int nlx, int ldx,
                                              const float2* __restrict__ Pj, const float2* __restrict__ tw,
                                              const int* __restrict__ band_h, const int* __restrict__ band_off,
                                              void* __restrict__ bcap, int64_t bstride, int sc, float2* lds) {
    using C = ColCfg<N>;
    constexpr int CW = C::CW, T = C::T, E = C::E;
    const int tid = threadIdx.x;
    const int strips = (ldx + CW - 1) / CW;
    const int64_t items = (int64_t)nbeam * strips;
    const int col = tid % CW, t = tid / CW;
    // Items (beam, strip), it = beam * strips + strip, are walked in chunks of gridDim.x; the
    // next chunk's strip is loaded while the current one is transformed.  Within a chunk the
    // 8 XCDs (block b runs on XCD b % 8) each take one contiguous range of items, so the
    // neighbouring strips that share 128-byte lines of a beam's rows run on one L2.
    const int G = gridDim.x, b = blockIdx.x;
    const int64_t slot = (G % 8 == 0) ? (int64_t)(b % 8) * (G / 8) + b / 8 : b;
    float2 nxt[E];
    auto load = [&](int64_t it) {
        const int64_t beam = it / strips;
        const int pc = (int)(it % strips) * CW + col;
        const bool live = logical_of_phys(pc, nlx, ldx) >= 0;
        const float2* plane = state + beam * (int64_t)N * ldx;
#pragma unroll
        for (int m = 0; m < E; ++m) nxt[m] = live ? plane[(int64_t)(t + T * m) * ldx + pc] : make_float2(0.f, 0.f);
    };
    const float2* __restrict__ px = Pj;         // column factors of the propagator
    const float2* __restrict__ py = Pj + nlx;   // row factors
    if (slot < items) load(slot);
    for (int64_t base = 0; base + slot < items; base += G) {
        const int64_t it = base + slot;
        float2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = nxt[m];
        const int64_t beam = it / strips;
        const int pc = (int)(it % strips) * CW + col;  // physical column (state)
        const int c = logical_of_phys(pc, nlx, ldx);   // live column (P, band tables)
        const bool live = c >= 0;
        const int h = live ? band_h[c] : -1;
        const float2 pxc = live ? px[c] : make_float2(0.f, 0.f);
        float2* plane = state + beam * (int64_t)N * ldx;
        if (it + G < items) load(it + G);
        constexpr int S1 = (MODE == 1 || MODE == 3) ? +1 : -1;   // first transform's sign (-1: FFT_y)
        fft_reg<N, S1, true>(v, lds, col, CW, t, tw);
#pragma unroll
        for (int m = 0; m < E; ++m) {
            const int ys = signed_index(t + T * m, N);
            float2 pv = (ys <= h && -ys <= h) ? cmul(pxc, py[t + T * m]) : make_float2(0.f, 0.f);
            if constexpr (MODE == 2 || MODE == 3) pv.y = -pv.y;   // inverse multislice: conj(P)
            v[m] = cmul(v[m], pv);
        }
        if (CAP && live) {
            // band coefficients of this column: ky = 0..h, then ny-h..ny-1, at band_off[c] + rank
            const int h = band_h[c];
            const int64_t dst = beam * bstride + band_off[c];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                int ky = t + T * m;
                int r = ky <= h ? ky : (ky >= N - h ? 2 * h + 1 - (N - ky) : -1);
                if (r >= 0) store_c(bcap, dst + r, v[m], sc);
            }
        }
        fft_reg<N, -S1, true>(v, lds, col, CW, t, tw);
        if (live) {
#pragma unroll
            for (int m = 0; m < E; ++m) plane[(int64_t)(t + T * m) * ldx + pc] = v[m];
        }
    }
}

template <int N, int MODE>
__global__ __launch_bounds__(ColCfg<N>::NT) __attribute__((amdgpu_waves_per_eu(RegCfg<N>::E > 16 ? 1 : 2))) void k_col_pass(
    float2* __restrict__ state, int nbeam, int nlx, int ldx, const float2* __restrict__ Pj,
    const float2* __restrict__ tw, const int* __restrict__ band_h) {
    __shared__ float2 lds[PadLen<N>::value * ColCfg<N>::CW];
    col_pass_body<N, MODE, false>(state, nbeam, nlx, ldx, Pj, tw, band_h, nullptr, nullptr, 0, 0, lds);
}

template <int N, int MODE>
__global__ __launch_bounds__(ColCfg<N>::NT) void k_col_pass_cap(float2* __restrict__ state, int nbeam, int nlx, int ldx,
                                                                const float2* __restrict__ Pj,
                                                                const float2* __restrict__ tw,
                                                                const int* __restrict__ band_h,
                                                                const int* __restrict__ band_off,
                                                                void* __restrict__ bcap, int64_t bstride, int sc) {
    __shared__ float2 lds[PadLen<N>::value * ColCfg<N>::CW];
    col_pass_body<N, MODE, true>(state, nbeam, nlx, ldx, Pj, tw, band_h, band_off, bcap, bstride, sc, lds);
}

// Band coefficients of P_{nz-1} e_q (the transposed sweep's start): P(q) at q's band slot.
__global__ void k_init_band(void* bcap, int64_t bstride, int Kb, const int4* beams, int nb, const int* band_h,
                            const int* band_off, int ny, int f, double lx, double ly, double lam, double dz_last,
                            int sc) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nb * bstride) return;
    int g = (int)(i % bstride);
    int b = (int)(i / bstride);
    int4 bm = beams[b];
    int h = band_h[bm.x];
    int r = bm.y <= h ? bm.y : 2 * h + 1 - (ny - bm.y);
    float2 v = make_float2(0.f, 0.f);
    if (g < Kb && g == band_off[bm.x] + r) {
        double kx = (double)(f * bm.z) / lx, ky = (double)(f * bm.w) / ly;
        double s, co;
        sincospi(-lam * dz_last * (kx * kx + ky * ky), &s, &co);
        v = make_float2((float)co, (float)s);
    }
    store_c(bcap, i, v, sc);
}

// Band FFT, row stage: rows y of T_j * W_i (real space, planes of `wstride` complex) times
// each transition potential H_t -> FFT_x -> live columns into scratch [(t Ni + i) ny + y][nlx].
// A thread group loads its row of W_i and T_j once and loops over the nt transitions (their
// H rows stay in L2), so the S_1 window is read once per site instead of once per transition.
// Row groups are walked with stride gridDim.x, the next group's W rows loaded meanwhile.
template <int N>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_band_rows(float2* __restrict__ out, const float2* __restrict__ W,
                                                   int64_t wstride, int Ni, int nt, int ny, int nlx, int hlx, int ldx,
                                                   const float2* __restrict__ Tj, const float2* __restrict__ Hb,
                                                   int64_t hstride, const float2* __restrict__ tw) {
    constexpr int E = RegCfg<N>::E, T = RegCfg<N>::T, S = 256 / T, L = PadLen<N>::value;
    __shared__ float2 lds[S * L];
    const int tid = threadIdx.x, s = tid / T, t = tid % T;
    const int64_t rows = (int64_t)Ni * ny;
    const int64_t ngroups = (rows + S - 1) / S;
    float2 nxt[E];
    auto load = [&](int64_t grp) {
        const int64_t g = grp * S + s;
        const bool ok = g < rows;
        const float2* wr = W + (ok ? (g / ny) * wstride + (g % ny) * N : 0);
#pragma unroll
        for (int m = 0; m < E; ++m) nxt[m] = ok ? wr[t + T * m] : make_float2(0.f, 0.f);
    };
    if ((int64_t)blockIdx.x < ngroups) load(blockIdx.x);
    for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
        const int64_t g = grp * S + s;
        const bool valid = g < rows;
        const int y = valid ? (int)(g % ny) : 0;
        const int i = valid ? (int)(g / ny) : 0;
        const float2* trow = Tj + (int64_t)y * N;
        float2 u[E];
#pragma unroll
        for (int m = 0; m < E; ++m) u[m] = valid ? cmul(nxt[m], trow[t + T * m]) : make_float2(0.f, 0.f);
        if (grp + gridDim.x < ngroups) load(grp + gridDim.x);
        // the next transition's H row is loaded while this one is transformed
        float2 h[E];
#pragma unroll
        for (int m = 0; m < E; ++m) h[m] = valid ? Hb[(int64_t)y * N + t + T * m] : make_float2(0.f, 0.f);
        for (int tt = 0; tt < nt; ++tt) {
            float2 v[E];
#pragma unroll
            for (int m = 0; m < E; ++m) v[m] = cmul(u[m], h[m]);
            if (tt + 1 < nt) {
                const float2* hr = Hb + (tt + 1) * hstride + (int64_t)y * N;
#pragma unroll
                for (int m = 0; m < E; ++m) h[m] = valid ? hr[t + T * m] : make_float2(0.f, 0.f);
            }
            fft_reg<N, -1, true, true>(v, lds, s * L, 1, t, tw);
            const int64_t o = (((int64_t)tt * Ni + i) * ny + y) * ldx;
#pragma unroll
            for (int m = 0; m < E; ++m) {
                int c = phys_col_of(t + T * m, N, hlx, ldx);
                if (valid && c >= 0) out[o + c] = v[m];
            }
        }
    }
}

// Band FFT, column stage: FFT_y of live-column strips, band coefficients to
// dst[plane * dstride + g] (SC or complex64); the padding slots Kb .. dstride-1 are zeroed.
// Items (plane, strip) are walked with stride gridDim.x, the next strip loaded meanwhile.
template <int N>
__global__ __launch_bounds__(ColCfg<N>::NT) __attribute__((amdgpu_waves_per_eu(2))) void k_band_cols(void* __restrict__ dst, int64_t dstride, int Kb,
                                                             const float2* __restrict__ src, int64_t n_planes,
                                                             int nlx, int ldx, const int* __restrict__ band_h,
                                                             const int* __restrict__ band_off,
                                                             const float2* __restrict__ tw, int sc) {
    using C = ColCfg<N>;
    constexpr int CW = C::CW, T = C::T, E = C::E, NT = C::NT;
    __shared__ float2 lds[PadLen<N>::value * CW];
    const int tid = threadIdx.x;
    const int strips = (ldx + CW - 1) / CW;
    const int64_t items = n_planes * strips;
    const int col = tid % CW, t = tid / CW;
    float2 nxt[E];
    auto load = [&](int64_t it) {
        const int pc = (int)(it % strips) * CW + col;
        const bool live = logical_of_phys(pc, nlx, ldx) >= 0;
        const float2* sp = src + (it / strips) * (int64_t)N * ldx;
#pragma unroll
        for (int m = 0; m < E; ++m) nxt[m] = live ? sp[(int64_t)(t + T * m) * ldx + pc] : make_float2(0.f, 0.f);
    };
    if ((int64_t)blockIdx.x < items) load(blockIdx.x);
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        float2 v[E];
#pragma unroll
        for (int m = 0; m < E; ++m) v[m] = nxt[m];
        const int64_t plane = it / strips;
        const int strip = (int)(it % strips);
        const int pc = strip * CW + col;
        const int c = logical_of_phys(pc, nlx, ldx);
        const bool live = c >= 0;
        if (it + gridDim.x < items) load(it + gridDim.x);
        fft_reg<N, -1, true>(v, lds, col, CW, t, tw);
        if (live) {
            const int h = band_h[c];
            const int64_t o = plane * dstride + band_off[c];
#pragma unroll
            for (int m = 0; m < E; ++m) {
                int ky = t + T * m;
                int r = ky <= h ? ky : (ky >= N - h ? 2 * h + 1 - (N - ky) : -1);
                if (r >= 0) store_c(dst, o + r, v[m], sc);
            }
        }
        if (strip == 0)
            for (int g = Kb + tid; g < dstride; g += NT) store_c(dst, plane * dstride + g, make_float2(0.f, 0.f), sc);
    }
}

// X[t][i][k] = H_t[k] * W_i[k] for k < K (zero for K <= k < ld), stored SC or complex64.
// X[(t Ni + r) ld + k] = H_t[k] W_r[k] for k < K, zero for K <= k < ld (ld a multiple of 4,
// X 32-byte aligned).  A block covers 1024 slots of one row r, 4 per thread: W_r is read
// once and the thread writes the nt transitions' products (H stays in cache), as whole
// 32-byte SC groups (or two complex64 pairs).
__global__ __launch_bounds__(256) void k_hmul(void* __restrict__ X, const float2* __restrict__ W, int64_t wstride,
                                              const float2* __restrict__ Hb, int64_t hstride, int Ni, int nt, int K,
                                              int ld, int sc, int xblocks) {
    const int r = (int)(blockIdx.x / xblocks);
    const int k0 = (int)(blockIdx.x % xblocks) * 1024 + 4 * threadIdx.x;
    if (k0 >= ld) return;
    const float2* w = W + r * wstride;
    float2 wv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) wv[e] = k0 + e < K ? w[k0 + e] : make_float2(0.f, 0.f);
    for (int t = 0; t < nt; ++t) {
        const float2* h = Hb + t * hstride;
        float2 v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = k0 + e < K ? cmul(h[k0 + e], wv[e]) : make_float2(0.f, 0.f);
        const int64_t off = ((int64_t)t * Ni + r) * ld + k0;
        if (sc == 0) {
            float4* o = (float4*)((float2*)X + off);
            o[0] = make_float4(v[0].x, v[0].y, v[1].x, v[1].y);
            o[1] = make_float4(v[2].x, v[2].y, v[3].x, v[3].y);
        } else {
            uint4 hi, lo;
            split_c(v[0], sc, hi.x, lo.x);
            split_c(v[1], sc, hi.y, lo.y);
            split_c(v[2], sc, hi.z, lo.z);
            split_c(v[3], sc, hi.w, lo.w);
            uint4* o = (uint4*)((uint32_t*)X + (off >> 2) * 8);
            o[0] = hi;
            o[1] = lo;
        }
    }
}

// --------------------------------------------------------------------- deterministic reduction
//
// map[R] += scale * sum over the CSR entries (desc, column i) of R of
//           sum_{tiles mt} sum_{t} part[p_off + mt ld_part + t N_inner + i]   (fixed order)
__global__ void k_reduce(double* map, int P, const int* __restrict__ rptr, const int2* __restrict__ ent,
                         const GemmDesc* __restrict__ descs, const float* __restrict__ part, double scale) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P) return;
    double acc = 0.0;
    for (int e = rptr[r]; e < rptr[r + 1]; ++e) {
        int2 en = ent[e];
        const GemmDesc& d = descs[en.x];
        const float* pp = part + d.p_off + en.y;
        for (int mt = 0; mt < d.tiles_m; ++mt)
            for (int t = 0; t < d.n_t; ++t) acc += (double)pp[(int64_t)mt * d.ld_part + (int64_t)t * d.N_inner];
    }
    map[r] += scale * acc;
}

// Dense form: every descriptor of the range covers every probe, column i = probe index.
__global__ void k_reduce_dense(double* map, int P, const GemmDesc* __restrict__ descs, int d_begin, int d_count,
                               const float* __restrict__ part, double scale) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P) return;
    double acc = 0.0;
    for (int e = 0; e < d_count; ++e) {
        const GemmDesc& d = descs[d_begin + e];
        const float* pp = part + d.p_off + r;
        for (int mt = 0; mt < d.tiles_m; ++mt)
            for (int t = 0; t < d.n_t; ++t) acc += (double)pp[(int64_t)mt * d.ld_part + (int64_t)t * d.N_inner];
    }
    map[r] += scale * acc;
}

// --------------------------------------------------------------------- launchers

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_twiddles(float2* tw, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_twiddles, dim3(blocks_for(n, 256)), dim3(256), 0, st, tw, n);
}
void launch_transmission(float2* T, const float* V, int64_t n, double sigma, hipStream_t st) {
    hipLaunchKernelGGL(k_transmission, dim3(blocks_for(n, 256)), dim3(256), 0, st, T, V, n, sigma);
}
void launch_propagator(float2* P, const double* dz, const Plan& p, hipStream_t st) {
    int64_t n = (int64_t)p.nz * (p.nlx + p.ny);
    hipLaunchKernelGGL(k_propagator, dim3(blocks_for(n, 256)), dim3(256), 0, st, P, dz, p.nz, p.nx, p.ny, p.nlx, p.hlx,
                       p.lx, p.ly, p.lam);
}
void launch_probe_coefficients(void* C, const int4* beams, const double* probes, const Plan& p, int sc,
                               hipStream_t st, int n_probes) {
    const int np = n_probes < 0 ? p.P : n_probes;
    int64_t n = (int64_t)np * p.N1pad;
    double scale = (double)p.f * p.f / std::sqrt((double)p.N1fine) * p.c_scale;
    hipLaunchKernelGGL(k_probe_coefficients, dim3(blocks_for(n, 256)), dim3(256), 0, st, C, beams, p.N1, p.N1pad,
                       probes, np, p.f, p.lx, p.ly, p.lam, p.defocus, p.cs, scale, sc);
}
void launch_init_forward(float2* S, const int4* beams, const Plan& p, hipStream_t st) {
    int64_t n = (int64_t)p.N1 * p.ny * p.nlx;
    hipLaunchKernelGGL(k_init_forward, dim3(blocks_for(n, 256)), dim3(256), 0, st, S, beams, p.N1, p.ny, p.nlx, p.ldx);
}
void launch_init_reverse(float2* S, const int4* beams, const Plan& p, hipStream_t st) {
    int64_t n = (int64_t)p.N2 * p.ny * p.nlx;
    hipLaunchKernelGGL(k_init_reverse, dim3(blocks_for(n, 256)), dim3(256), 0, st, S, beams, p.N2, p.ny, p.nlx, p.ldx, p.f,
                       p.lx, p.ly, p.lam, p.dz[p.nz - 1]);
}
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t st) {
    int64_t n4 = (int64_t)(bytes / 16);
    if (n4 <= 0) return;
    int64_t blocks = std::min<int64_t>(blocks_for(n4, 256), 65536);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (float4*)ptr, n4);
}
void launch_fill_zero_d(double* p, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_zero_d, dim3(blocks_for(n, 256)), dim3(256), 0, st, p, n);
}
void launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 256)), dim3(256), 0, st, dst, src, n);
}

// Grid of the block-strided pass kernels: every block walks several items so that its
// register prefetch overlaps; 2048 blocks (8 per CU) balance the tail.
static inline unsigned strided_grid(int64_t items) { return (unsigned)std::min<int64_t>(items, 2048); }

template <int N, int MODE>
static void row_pass_n(const RowPassArgs& a, hipStream_t st) {
    constexpr int S = 256 / RegCfg<N>::T;
    int64_t rows = (int64_t)a.nbeam * a.ny;
    if (rows <= 0) return;
    const dim3 grid(strided_grid(blocks_for(rows, S)));
    if (a.cap_ptr)
        hipLaunchKernelGGL((k_row_pass_cap<N, MODE>), grid, dim3(256), 0, st, a.state, a.nbeam, a.ny, a.nlx, a.hlx,
                           a.ldx, a.Tj, a.tw, a.cap_ptr, (const int4*)a.cap_rec, a.win, a.win_beams, a.Kpad, a.sc,
                           a.cfac);
    else
        hipLaunchKernelGGL((k_row_pass<N, MODE>), grid, dim3(256), 0, st, a.state, a.nbeam, a.ny, a.nlx, a.hlx, a.ldx,
                           a.Tj, a.tw);
}

void launch_row_pass(int nx, int mode, const RowPassArgs& a, hipStream_t st) {
#define ROWCASE(NN)                                   \
    case NN:                                          \
        if (mode == 0) row_pass_n<NN, 0>(a, st);      \
        else if (mode == 1) row_pass_n<NN, 1>(a, st); \
        else if (mode == 2) row_pass_n<NN, 2>(a, st); \
        else if (mode == 3) row_pass_n<NN, 3>(a, st); \
        else row_pass_n<NN, 4>(a, st);                \
        break;
    switch (nx) {
        ROWCASE(16) ROWCASE(32) ROWCASE(64) ROWCASE(128) ROWCASE(256) ROWCASE(384) ROWCASE(512) ROWCASE(1024)
        default: break;
    }
#undef ROWCASE
}

template <int N, int MODE>
static void col_pass_n(float2* state, int nbeam, int nlx, int ldx, const float2* Pj, const float2* tw,
                       const int* band_h, const BandCap& bc, hipStream_t st) {
    using C = ColCfg<N>;
    int strips = (ldx + C::CW - 1) / C::CW;
    if (nbeam <= 0) return;
    const dim3 grid(strided_grid((int64_t)nbeam * strips));
    if (bc.dst)
        hipLaunchKernelGGL((k_col_pass_cap<N, MODE>), grid, dim3(C::NT), 0, st, state, nbeam, nlx, ldx, Pj, tw,
                           band_h, bc.band_off, bc.dst, bc.stride, bc.sc);
    else
        hipLaunchKernelGGL((k_col_pass<N, MODE>), grid, dim3(C::NT), 0, st, state, nbeam, nlx, ldx, Pj, tw, band_h);
}

void launch_col_pass(int ny, int mode, float2* state, int nbeam, int nlx, int ldx, const float2* Pj, const float2* tw,
                     const int* band_h, const BandCap& bc, hipStream_t st) {
#define COLCASE(NN)                                                   \
    case NN:                                                          \
        if (mode == 0) col_pass_n<NN, 0>(state, nbeam, nlx, ldx, Pj, tw, band_h, bc, st); \
        else if (mode == 1) col_pass_n<NN, 1>(state, nbeam, nlx, ldx, Pj, tw, band_h, bc, st); \
        else if (mode == 2) col_pass_n<NN, 2>(state, nbeam, nlx, ldx, Pj, tw, band_h, bc, st); \
        else col_pass_n<NN, 3>(state, nbeam, nlx, ldx, Pj, tw, band_h, bc, st);    \
        break;
    switch (ny) {
        COLCASE(16) COLCASE(32) COLCASE(64) COLCASE(128) COLCASE(256) COLCASE(384) COLCASE(512) COLCASE(1024)
        default: break;
    }
#undef COLCASE
}

void launch_init_band(void* bcap, int64_t bstride, const int4* beams, const int* band_h, const int* band_off,
                      const Plan& p, int sc, hipStream_t st) {
    int64_t n = (int64_t)p.N2 * bstride;
    hipLaunchKernelGGL(k_init_band, dim3(blocks_for(n, 256)), dim3(256), 0, st, bcap, bstride, p.Kb, beams, p.N2,
                       band_h, band_off, p.ny, p.f, p.lx, p.ly, p.lam, p.dz[p.nz - 1], sc);
}

template <int NX, int NY>
static void band_fft_n(const BandFft& a, hipStream_t st) {
    constexpr int S = 256 / RegCfg<NX>::T;
    int64_t rows = (int64_t)a.Ni * a.ny;
    hipLaunchKernelGGL((k_band_rows<NX>), dim3(strided_grid(blocks_for(rows, S))), dim3(256), 0, st, a.scratch, a.W,
                       a.wstride, a.Ni, a.nt, a.ny, a.nlx, a.hlx, a.ldx, a.Tj, a.H, a.hstride, a.twx);
    using C = ColCfg<NY>;
    int strips = (a.ldx + C::CW - 1) / C::CW;
    const int64_t planes = (int64_t)a.nt * a.Ni;
    hipLaunchKernelGGL((k_band_cols<NY>), dim3(strided_grid(planes * strips)), dim3(C::NT), 0, st, a.dst, a.dstride,
                       a.Kb, a.scratch, planes, a.nlx, a.ldx, a.band_h, a.band_off, a.twy, a.sc);
}

void launch_band_fft(int nx, int ny, const BandFft& a, hipStream_t st) {
    if ((int64_t)a.nt * a.Ni <= 0) return;
#define BF(X)                                              \
    case X:                                                \
        switch (nx) {                                      \
            case 16: band_fft_n<16, X>(a, st); break;     \
            case 32: band_fft_n<32, X>(a, st); break;     \
            case 64: band_fft_n<64, X>(a, st); break;     \
            case 128: band_fft_n<128, X>(a, st); break;   \
            case 256: band_fft_n<256, X>(a, st); break;   \
            case 512: band_fft_n<512, X>(a, st); break;   \
            case 1024: band_fft_n<1024, X>(a, st); break; \
        }                                                  \
        break;
    switch (ny) { BF(16) BF(32) BF(64) BF(128) BF(256) BF(512) BF(1024) }
#undef BF
}

template <int NX>
static void band_rows_n(float2* out, const float2* W, int64_t wstride, int Ni, int nt, const Plan& p,
                        const float2* Tj, const float2* H, int64_t hstride, const float2* tw, hipStream_t st) {
    constexpr int S = 256 / RegCfg<NX>::T;
    int64_t rows = (int64_t)Ni * p.ny;
    hipLaunchKernelGGL((k_band_rows<NX>), dim3(strided_grid(blocks_for(rows, S))), dim3(256), 0, st, out, W, wstride,
                       Ni, nt, p.ny, p.nlx, p.hlx, p.ldx, Tj, H, hstride, tw);
}

void launch_band_rows(float2* out, const float2* W, int64_t wstride, int Ni, int nt, const Plan& p, const float2* Tj,
                      const float2* H, int64_t hstride, const float2* tw, hipStream_t st) {
    if ((int64_t)Ni * nt <= 0) return;
    switch (p.nx) {
        case 16: band_rows_n<16>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 32: band_rows_n<32>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 64: band_rows_n<64>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 128: band_rows_n<128>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 256: band_rows_n<256>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 512: band_rows_n<512>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        case 1024: band_rows_n<1024>(out, W, wstride, Ni, nt, p, Tj, H, hstride, tw, st); break;
        default: break;
    }
}

void launch_hmul(void* X, const float2* W, int64_t wstride, const float2* H, int64_t hstride, int Ni, int nt, int K,
                 int ld, int sc, hipStream_t st) {
    if ((int64_t)nt * Ni <= 0 || ld <= 0) return;
    const int xblocks = (int)ceil_div(ld, 1024);
    hipLaunchKernelGGL(k_hmul, dim3((unsigned)((int64_t)Ni * xblocks)), dim3(256), 0, st, X, W, wstride, H, hstride, Ni,
                       nt, K, ld, sc, xblocks);
}

void launch_reduce(double* map, int P, const int* rptr, const int* ent, const GemmDesc* descs, const float* part,
                   double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(blocks_for(P, 256)), dim3(256), 0, st, map, P, rptr, (const int2*)ent, descs,
                       part, scale);
}
void launch_reduce_dense(double* map, int P, const GemmDesc* descs, int d_begin, int d_count, const float* part,
                         double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_dense, dim3(blocks_for(P, 256)), dim3(256), 0, st, map, P, descs, d_begin, d_count,
                       part, scale);
}

}  // namespace eels
