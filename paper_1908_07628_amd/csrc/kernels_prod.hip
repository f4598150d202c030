// Producers of the split GEMM operands and the window-Gram detector sum: SC conversions, the
// window transposes (with the SC copy of the S_1 window in the raster form), G = M o sum_t
// conj(H_t) H_t^T and the per-probe dot products.  All HBM-bound: each moves its operands once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fft_lds.h"
#include "internal.h"
#include "kernels.h"
#include "sc_format.h"
#include "stream_store.h"

namespace eels {

// complex64 -> SC conversion of rows [rows][ld] (K padding columns become zero); batched: job
// blockIdx.y's S_1 window (s1w) into its s1sc slot
__global__ void k_to_sc(uint32_t* __restrict__ dst, const float2* __restrict__ src, int64_t rows, int K, int ld,
                        int prec, const ProdJob* __restrict__ jobs) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * ld) return;
    if (jobs) {
        const ProdJob& j = jobs[blockIdx.y];
        src += j.s1w;
        dst = (uint32_t*)((char*)dst + 8 * j.s1sc);
    }
    int k = (int)(i % ld);
    float2 v = k < K ? src[i] : make_float2(0.f, 0.f);
    sc_store(dst, i, v, prec);
}

// Window transpose for the order-P products: the window [beam][pixel] (complex64, rows
// wstride apart) becomes rows [pixel][beam] of ldo complex, beams n_beams .. ldo-1 zero;
// split precisions store SC rows (the B operand of the split probe-wave product Psi = C S_1w,
// or of the window-Gram form's Gram GEMM), FP32 complex64 rows.  A block moves a 64-pixel x
// 64-beam tile through LDS, reading whole pixel runs of a beam and writing whole 4-beam
// groups of a pixel.
// x = hi + lo from an SC pair (hi and lo: (re, im) half pairs of one complex slot)
__device__ __forceinline__ float2 sc_value(uint32_t hi, uint32_t lo, int prec) {
    if (prec == EELS_BF16_SPLIT)
        return make_float2(__uint_as_float(hi << 16) + __uint_as_float(lo << 16),
                           __uint_as_float(hi & 0xffff0000u) + __uint_as_float(lo & 0xffff0000u));
    const _Float16 hr = __builtin_bit_cast(_Float16, (uint16_t)(hi & 0xffffu));
    const _Float16 hi2 = __builtin_bit_cast(_Float16, (uint16_t)(hi >> 16));
    const _Float16 lr = __builtin_bit_cast(_Float16, (uint16_t)(lo & 0xffffu));
    const _Float16 li = __builtin_bit_cast(_Float16, (uint16_t)(lo >> 16));
    return make_float2((float)hr + (float)lr, (float)hi2 + (float)li);
}

template <int PREC>
__global__ __launch_bounds__(256) void k_window_t_sc(uint32_t* __restrict__ dst, const float2* __restrict__ src,
                                                     int64_t wstride, int n_beams, int K, int ldo,
                                                     const int* __restrict__ perm, const ProdJob* __restrict__ jobs,
                                                     int which, int copy_prec, int copy_ld,
                                                     const float2* __restrict__ cph, int in_sc) {
    // The tile holds beam row r, pixel c at tile[r][c ^ ((r >> 2) & 15)].  The swizzle puts the
    // 16 rows 4g + e (g = 0 .. 15) that a quarter-wave reads for one pixel in 16 distinct 8-byte
    // bank pairs (a padded 65-slot row left 4 of them in each), keeps every 4-pixel group of a
    // row in one aligned 32-byte block, and permutes a row's pixels (conflict-free row writes).
    __shared__ __attribute__((aligned(16))) float2 tile[64][64];
    uint32_t* cp = nullptr;
    if (jobs) {   // batched: job blockIdx.z's window (which 0: S_2 -> s2t, 1: S_1 -> xt, 2: S_1 -> s2t)
        const ProdJob& j = jobs[blockIdx.z];
        src += which ? j.s1w : j.s2w;
        if (copy_prec) cp = (uint32_t*)((char*)dst + 8 * j.s1sc);
        dst = (uint32_t*)((char*)dst + 8 * (which == 1 ? j.xt : j.s2t));
    }
    const int p0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int b = b0 + r, px = p0 + tx;
        const int bs = (perm && b < n_beams) ? perm[b] : b;
        float2 v = make_float2(0.f, 0.f);
        if (b < n_beams && px < K) {
            const int64_t o = (int64_t)bs * wstride + px;
            if (in_sc) {
                const uint32_t* w = (const uint32_t*)src + (o >> 2) * 8 + (o & 3);
                v = sc_value(w[0], w[4], in_sc);
            } else {
                v = ld_stream(src + o);
            }
        }
        if (cph && b < n_beams) v = cmul(cph[bs], v);   // the beam's factor, folded into both outputs
        tile[r][tx ^ ((r >> 2) & 15)] = v;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < 64 * 16; w += 256) {
        const int px = w >> 4, g = w & 15;
        const int pix = p0 + px, b = b0 + 4 * g;
        if (pix >= K || b >= ldo) continue;
        const int pc = px ^ g;            // rows 4 g .. 4 g + 3 all swizzle by g
        if constexpr (PREC == EELS_FP32) {
            float4* o = (float4*)((float2*)dst + (int64_t)pix * ldo + b);
            const float2 v0 = tile[4 * g][pc], v1 = tile[4 * g + 1][pc], v2 = tile[4 * g + 2][pc],
                         v3 = tile[4 * g + 3][pc];
            st_stream(o, make_float4(v0.x, v0.y, v1.x, v1.y));
            st_stream(o + 1, make_float4(v2.x, v2.y, v3.x, v3.y));
        } else {
            u32x4 hi, lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float2 v = tile[4 * g + e][pc];
                uint32_t h, l;
                split2<PREC>(v.x, v.y, h, l);
                hi[e] = h;
                lo[e] = l;
            }
            uint32_t* o = dst + (((int64_t)pix * ldo + b) >> 2) * 8;
            st_stream_vec((u32x4*)o, hi);
            st_stream_vec((u32x4*)(o + 4), lo);
        }
    }
    if (cp) {
        // the same tile untransposed into the window's SC copy [beam][copy_ld] (the raster form's Z
        // GEMM operand): slot b's row goes back to beam perm[b], pixels K .. copy_ld - 1 are zero.
        // Pixels 4g .. 4g + 3 of row r sit in the aligned block 4 (g ^ (z >> 2)), z = (r >> 2) & 15,
        // pixel 4g + e at position e ^ (z & 3); a quarter-wave reads one row's 16 blocks.
        for (int w = threadIdx.x; w < 64 * 16; w += 256) {
            const int r = w >> 4, g = w & 15;
            const int b = b0 + r, px = p0 + 4 * g;
            if (b >= n_beams || px >= copy_ld) continue;
            const int bs = perm ? perm[b] : b;
            const int z = (r >> 2) & 15;
            const float4* blk = (const float4*)&tile[r][4 * (g ^ (z >> 2))];
            const float4 q0 = blk[0], q1 = blk[1];
            float2 v[4] = {make_float2(q0.x, q0.y), make_float2(q0.z, q0.w), make_float2(q1.x, q1.y),
                           make_float2(q1.z, q1.w)};
            if (z & 1) { const float2 a = v[0]; v[0] = v[1]; v[1] = a; const float2 c = v[2]; v[2] = v[3]; v[3] = c; }
            if (z & 2) { const float2 a = v[0]; v[0] = v[2]; v[2] = a; const float2 c = v[1]; v[1] = v[3]; v[3] = c; }
            u32x4 hi, lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t h, l;
                if (copy_prec == EELS_BF16_SPLIT) split2<EELS_BF16_SPLIT>(v[e].x, v[e].y, h, l);
                else split2<EELS_FP16_SPLIT>(v[e].x, v[e].y, h, l);
                hi[e] = h;
                lo[e] = l;
            }
            uint32_t* o = cp + (((int64_t)bs * copy_ld + px) >> 2) * 8;
            st_stream_vec((u32x4*)o, hi);
            st_stream_vec((u32x4*)(o + 4), lo);
        }
    }
}

static void window_t_go(void* dst, const float2* src, int64_t wstride, int n_beams, int K, int ldo, int prec,
                        hipStream_t st, const int* perm, const ProdJob* jobs, int n_jobs, int which, int copy_prec,
                        int copy_ld, const float2* cph, int in_sc = 0) {
    if (n_beams <= 0 || K <= 0 || n_jobs <= 0) return;
    dim3 grid((unsigned)ceil_div(K, 64), (unsigned)ceil_div(ldo, 64), (unsigned)n_jobs);
    if (prec == EELS_BF16_SPLIT)
        hipLaunchKernelGGL(k_window_t_sc<EELS_BF16_SPLIT>, grid, dim3(256), 0, st, (uint32_t*)dst, src, wstride,
                           n_beams, K, ldo, perm, jobs, which, copy_prec, copy_ld, cph, in_sc);
    else if (prec == EELS_FP16_SPLIT)
        hipLaunchKernelGGL(k_window_t_sc<EELS_FP16_SPLIT>, grid, dim3(256), 0, st, (uint32_t*)dst, src, wstride,
                           n_beams, K, ldo, perm, jobs, which, copy_prec, copy_ld, cph, in_sc);
    else
        hipLaunchKernelGGL(k_window_t_sc<EELS_FP32>, grid, dim3(256), 0, st, (uint32_t*)dst, src, wstride,
                           n_beams, K, ldo, perm, jobs, which, copy_prec, copy_ld, cph, in_sc);
}

void launch_window_t_sc(void* dst, const float2* src, int64_t wstride, int n_beams, int K, int ldo, int prec,
                        hipStream_t st, const int* perm) {
    window_t_go(dst, src, wstride, n_beams, K, ldo, prec, st, perm, nullptr, 1, 0, 0, 0, nullptr);
}

void launch_window_t_batched(void* dst_base, const float2* src_base, const ProdJob* jobs, int n_jobs, int which,
                             int64_t wstride, int n_beams, int K, int ldo, int prec, const int* perm, hipStream_t st,
                             int copy_prec, int copy_ld, const float2* cph, int in_sc) {
    window_t_go(dst_base, src_base, wstride, n_beams, K, ldo, prec, st, perm, jobs, n_jobs, which, copy_prec,
                copy_ld, cph, in_sc);
}

// zero complex slots K .. ld-1 of every SC row (a thread per row and padding slot)
__global__ void k_sc_zero_cols(uint32_t* __restrict__ base, int64_t rows, int ld, int K) {
    const int pad = ld - K;
    const int64_t n = rows * pad;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = (i / pad) * ld + K + (int)(i % pad);
        uint32_t* w = base + (o >> 2) * 8 + (o & 3);
        w[0] = 0u;
        w[4] = 0u;
    }
}

void launch_sc_zero_cols(void* base, int64_t rows, int ld, int K, hipStream_t st) {
    if (rows <= 0 || ld <= K) return;
    const int64_t n = rows * (ld - K);
    hipLaunchKernelGGL(k_sc_zero_cols, dim3((unsigned)std::min<int64_t>(ceil_div(n, 256), 8192)), dim3(256), 0, st,
                       (uint32_t*)base, rows, ld, K);
}

// Window-Gram form of the detector sum: G = gscale M o S with S[r][c] = sum_t conj(H_t[r]) H_t[c]
// (H_t the site's transition potentials on its K window pixels), written as SC rows
// [K][ldg] (columns K .. ldg-1 zero), or complex64 rows for FP32.  M holds FP32 complex Gram tiles [K][ldm] of the
// 128 x 128 grid with tile column >= tile row only; the others are the conjugate transpose.
// A block forms a 64 x 64 tile, both of whose 128-tiles are on one side of the diagonal,
// so it reads either M's tile or the transposed tile (through LDS), and stages the H values
// of its rows and columns 16 transitions at a time.
template <int PREC>
__global__ __launch_bounds__(256) void k_wgram_combine(uint32_t* __restrict__ dst, const float2* __restrict__ Mg,
                                                       const float2* __restrict__ H, int nt, int K, int ldm,
                                                       int ldg, float gscale, const ProdJob* __restrict__ jobs) {
    __shared__ float2 tile[64][65];
    if (jobs) {   // batched: job blockIdx.z's G, M (both in the buffer dst and Mg point to) and H
        const ProdJob& j = jobs[blockIdx.z];
        dst = (uint32_t*)((char*)dst + 8 * j.g);
        Mg += j.m;
        H += j.h;
        nt = j.nt;
    }
    __shared__ float2 hr[16][64], hc[16][64];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const bool mirror = (r0 >> 7) > (c0 >> 7);
    for (int a = ty; a < 64; a += 4) {
        if (!mirror) {
            const int r = r0 + a, c = c0 + tx;
            tile[a][tx] = (r < K && c < K) ? Mg[(int64_t)r * ldm + c] : make_float2(0.f, 0.f);
        } else {   // M(r, c) = conj(M(c, r)): read row c0 + a of M along r
            const int c = c0 + a, r = r0 + tx;
            const float2 v = (r < K && c < K) ? Mg[(int64_t)c * ldm + r] : make_float2(0.f, 0.f);
            tile[tx][a] = make_float2(v.x, -v.y);
        }
    }
    // each thread owns 4 rows x one 4-column group: rows ty + 4 j' (j' = 0..15 over 4 passes)
    float sr[4][4], si[4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) { sr[j][e] = 0.f; si[j][e] = 0.f; }
    const int g = threadIdx.x & 15, rb = threadIdx.x >> 4;   // column group, row base 0..15
    for (int t0 = 0; t0 < nt; t0 += 16) {
        __syncthreads();
        for (int w = threadIdx.x; w < 16 * 64; w += 256) {
            const int tt = w >> 6, x = w & 63;
            const bool ok = t0 + tt < nt;
            hr[tt][x] = (ok && r0 + x < K) ? H[(int64_t)(t0 + tt) * K + r0 + x] : make_float2(0.f, 0.f);
            hc[tt][x] = (ok && c0 + x < K) ? H[(int64_t)(t0 + tt) * K + c0 + x] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const int tn = min(16, nt - t0);
        for (int tt = 0; tt < tn; ++tt) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float2 a = hr[tt][rb + 16 * j];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const float2 b = hc[tt][4 * g + e];
                    sr[j][e] += a.x * b.x + a.y * b.y;     // conj(a) b
                    si[j][e] += a.x * b.y - a.y * b.x;
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int y = rb + 16 * j, r = r0 + y, c = c0 + 4 * g;
        if (r >= K || c >= ldg) continue;
        float vr[4], vi[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float2 m = tile[y][4 * g + e];
            vr[e] = gscale * (m.x * sr[j][e] - m.y * si[j][e]);
            vi[e] = gscale * (m.x * si[j][e] + m.y * sr[j][e]);
            if (c + e >= K) { vr[e] = 0.f; vi[e] = 0.f; }
        }
        if constexpr (PREC == EELS_FP32) {
            float4* o = (float4*)((float2*)dst + (int64_t)r * ldg + c);
            o[0] = make_float4(vr[0], vi[0], vr[1], vi[1]);
            o[1] = make_float4(vr[2], vi[2], vr[3], vi[3]);
        } else {
            u32x4 hi, lo;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t h, l;
                split2<PREC>(vr[e], vi[e], h, l);
                hi[e] = h;
                lo[e] = l;
            }
            uint32_t* o = dst + (((int64_t)r * ldg + c) >> 2) * 8;
            *(u32x4*)o = hi;
            *(u32x4*)(o + 4) = lo;
        }
    }
}

// Window-Gram form: out[i] = oscale sum_r Re(conj(Psi[i][r]) Y[i][r]) over the K window pixels,
// Psi in SC rows of ld complex (complex64 for FP32), Y complex64 rows of ld; one wave per
// probe row.
template <int PREC>
__global__ __launch_bounds__(256) void k_wgram_dot(float* __restrict__ out, const uint32_t* __restrict__ psi,
                                                   const float2* __restrict__ Y, int rows, int K, int ld,
                                                   float oscale) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= rows) return;
    const uint32_t* prow = psi + ((int64_t)i * ld >> 2) * 8;
    const float2* yrow = Y + (int64_t)i * ld;
    float acc = 0.f;
    if constexpr (PREC == EELS_FP32) {
        const float2* prow2 = (const float2*)psi + (int64_t)i * ld;
        for (int r = lane; r < K; r += 64) {
            const float2 a = prow2[r], y = yrow[r];
            acc += a.x * y.x + a.y * y.y;
        }
    } else
    for (int gi = lane; gi * 4 < K; gi += 64) {
        const u32x4 h = *(const u32x4*)(prow + 8 * gi);
        const u32x4 l = *(const u32x4*)(prow + 8 * gi + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = 4 * gi + e;
            if (r >= K) break;
            float pr, pi;
            if constexpr (PREC == EELS_BF16_SPLIT) {
                pr = __uint_as_float(h[e] << 16) + __uint_as_float(l[e] << 16);
                pi = __uint_as_float(h[e] & 0xFFFF0000u) + __uint_as_float(l[e] & 0xFFFF0000u);
            } else {
                pr = (float)__builtin_bit_cast(_Float16, (uint16_t)(h[e] & 0xFFFF)) +
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(l[e] & 0xFFFF));
                pi = (float)__builtin_bit_cast(_Float16, (uint16_t)(h[e] >> 16)) +
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(l[e] >> 16));
            }
            const float2 y = yrow[r];
            acc += pr * y.x + pi * y.y;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) out[i] = oscale * acc;
}

static void combine_go(void* G, const float2* M, const float2* H, int nt, int K, int ldm, int ldg, float gscale,
                       int prec, hipStream_t st, const ProdJob* jobs, int n_jobs) {
    if (K <= 0 || n_jobs <= 0) return;
    dim3 grid((unsigned)ceil_div(ldg, 64), (unsigned)ceil_div(K, 64), (unsigned)n_jobs);
    if (prec == EELS_BF16_SPLIT)
        hipLaunchKernelGGL(k_wgram_combine<EELS_BF16_SPLIT>, grid, dim3(256), 0, st, (uint32_t*)G, M, H, nt, K, ldm,
                           ldg, gscale, jobs);
    else if (prec == EELS_FP16_SPLIT)
        hipLaunchKernelGGL(k_wgram_combine<EELS_FP16_SPLIT>, grid, dim3(256), 0, st, (uint32_t*)G, M, H, nt, K, ldm,
                           ldg, gscale, jobs);
    else
        hipLaunchKernelGGL(k_wgram_combine<EELS_FP32>, grid, dim3(256), 0, st, (uint32_t*)G, M, H, nt, K, ldm,
                           ldg, gscale, jobs);
}

void launch_wgram_combine(void* G, const float2* M, const float2* H, int nt, int K, int ldm, int ldg, float gscale,
                          int prec, hipStream_t st) {
    combine_go(G, M, H, nt, K, ldm, ldg, gscale, prec, st, nullptr, 1);
}

void launch_wgram_combine_batched(void* mid2, const float2* H, const ProdJob* jobs, int n_jobs, int K, int ldm, int ldg,
                                  float gscale, int prec, hipStream_t st) {
    combine_go(mid2, (const float2*)mid2, H, 0, K, ldm, ldg, gscale, prec, st, jobs, n_jobs);
}

void launch_wgram_dot(float* out, const void* psi, const float2* Y, int rows, int K, int ld, float oscale, int prec,
                      hipStream_t st) {
    if (rows <= 0) return;
    dim3 grid((unsigned)ceil_div(rows, 4));
    if (prec == EELS_BF16_SPLIT)
        hipLaunchKernelGGL(k_wgram_dot<EELS_BF16_SPLIT>, grid, dim3(256), 0, st, out, (const uint32_t*)psi, Y, rows,
                           K, ld, oscale);
    else if (prec == EELS_FP16_SPLIT)
        hipLaunchKernelGGL(k_wgram_dot<EELS_FP16_SPLIT>, grid, dim3(256), 0, st, out, (const uint32_t*)psi, Y, rows,
                           K, ld, oscale);
    else
        hipLaunchKernelGGL(k_wgram_dot<EELS_FP32>, grid, dim3(256), 0, st, out, (const uint32_t*)psi, Y, rows,
                           K, ld, oscale);
}

__global__ void k_from_sc(float2* __restrict__ dst, const uint32_t* __restrict__ src, int64_t n, int prec) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t u = i >> 2;
    int pos = (int)(i & 3);
    uint32_t h = src[u * 8 + pos], l = src[u * 8 + 4 + pos];
    float2 v;
    if (prec == EELS_BF16_SPLIT) {
        v.x = __uint_as_float(h << 16) + __uint_as_float(l << 16);
        v.y = __uint_as_float(h & 0xFFFF0000u) + __uint_as_float(l & 0xFFFF0000u);
    } else {
        v.x = (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xFFFF)) + (float)__builtin_bit_cast(_Float16, (uint16_t)(l & 0xFFFF));
        v.y = (float)__builtin_bit_cast(_Float16, (uint16_t)(h >> 16)) + (float)__builtin_bit_cast(_Float16, (uint16_t)(l >> 16));
    }
    dst[i] = v;
}

void launch_from_sc(float2* dst, const void* src, int64_t n, int prec, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_from_sc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, (const uint32_t*)src, n, prec);
}

void launch_to_sc(void* dst, const float2* src, int64_t rows, int K, int ld, int prec, hipStream_t st) {
    int64_t n = rows * ld;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_to_sc, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (uint32_t*)dst, src, rows, K, ld,
                       prec, (const ProdJob*)nullptr);
}

void launch_to_sc_batched(void* dst_base, const float2* src_base, const ProdJob* jobs, int n_jobs, int64_t rows, int K,
                          int ld, int prec, hipStream_t st) {
    int64_t n = rows * ld;
    if (n <= 0 || n_jobs <= 0) return;
    hipLaunchKernelGGL(k_to_sc, dim3((unsigned)((n + 255) / 256), (unsigned)n_jobs), dim3(256), 0, st,
                       (uint32_t*)dst_base, src_base, rows, K, ld, prec, jobs);
}

}  // namespace eels
