// Grouped complex GEMM on the CDNA4 matrix cores for the contractions of Eq. SHn0:
//     C[m][n] = sum_k A[m][k] * B[n][k]              (no conjugation)
// with an optional transition-potential prologue on B (B[n][k] *= H_t[k], Eq. Hn0Psi)
// and either a plain store or a |C|^2 column-sum epilogue (the detector sum).
//
// Complex products without complex MFMA: with A' = (Ar, Ai) interleaved along k, the
// real and imaginary parts are the real products
//     Re C = A' . (Br, -Bi),   Im C = A' . (Bi, Br)
// so complex data stays interleaved in memory and each lane builds its B operand with
// a sign flip and a swap.  FP32 uses v_mfma_f32_32x32x2_f32 (one complex k per
// instruction).  The split precisions store x = hi + lo (hi = rn(x), lo = rn(x - hi))
// in bf16 or fp16 and use v_mfma_f32_32x32x16 (eight complex k per instruction) for
// hi*hi + hi*lo + lo*hi with fp32 accumulation.
//
// Block: 256 threads = 4 waves in a 2 x 2 grid over a 128 x 128 complex output tile;
// each wave owns 64 x 64 = 2 x 2 MFMA blocks of 32 x 32.  K advances 16 complex per
// step through LDS with the next step's global loads issued before the MFMAs.  The split
// kernel also has a 512-thread form, 8 waves in a 4 x 2 grid over a 256 x 128 tile, for
// the store epilogue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "internal.h"
#include "kernels.h"
#include "sc_format.h"

namespace eels {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = 16;
constexpr int LDF = BK + 1;   // float2 row stride of single-precision tiles
constexpr int LDS_ = BK + 4;  // u32 row stride of split tiles (one u32 = one complex half pair)

__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int PREC>
__device__ __forceinline__ floatx16 mfma16(u32x4 a, u32x4 b, floatx16 c) {
    if constexpr (PREC == EELS_BF16_SPLIT)
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                       0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(halfx8, a), __builtin_bit_cast(halfx8, b), c,
                                                      0, 0, 0);
}

__device__ __forceinline__ u32x4 neg_imag(u32x4 v) {  // (re, im) -> (re, -im) per half pair
    return v ^ (u32x4){0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
}
__device__ __forceinline__ u32x4 swap_halves(u32x4 v) {  // (re, im) -> (im, re)
    return (v >> 16) | (v << 16);
}

// Block -> (descriptor, m tile, n tile, t).  Tile orders within a descriptor and t:
//   0  m fastest (the blocks in flight share B tiles)
//   1  n fastest (they share A tiles)
//   2  XCD-aware: workgroups are dispatched to the 8 XCDs round-robin, so block b runs
//      on XCD b % 8; each XCD is given one contiguous range of tiles, walked in groups of
//      8 m tiles with m fastest, so the blocks resident on one XCD cover a compact
//      8 x 8 patch of the output and its L2 holds only their A and B rows.
// Returns the descriptor index.
template <int G = 8>
__device__ __forceinline__ int locate_tile(const GemmDesc* __restrict__ descs, int n_desc, int order, int& tm,
                                           int& tn, int& t, int bid, int ntiles) {
    if (order == 2) {
        const int nt = ntiles, x = bid & 7, s = bid >> 3, q = nt >> 3, r = nt & 7;
        bid = x * q + min(x, r) + s;
    }
    int lo = 0, hi = n_desc - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (descs[mid].tile_start <= bid) lo = mid;
        else hi = mid - 1;
    }
    const GemmDesc& d = descs[lo];
    const int local = bid - d.tile_start;
    const int per_t = d.tiles_m * d.tiles_n;
    t = local / per_t;
    const int r = local - t * per_t;
    if (order == 1) {
        tn = r % d.tiles_n;
        tm = r / d.tiles_n;
    } else if (order == 0) {
        tm = r % d.tiles_m;
        tn = r / d.tiles_m;
    } else {
        const int grp = r / (G * d.tiles_n), fm = grp * G;
        const int gs = min(d.tiles_m - fm, G);
        const int w = r - grp * G * d.tiles_n;
        tm = fm + w % gs;
        tn = w / gs;
    }
    return lo;
}

template <int PREC, int KIND, int EPI>
__global__ __launch_bounds__(256) void k_cgemm(const GemmDesc* __restrict__ descs, int n_desc,
                                               const float2* __restrict__ Ab, const float2* __restrict__ Bb,
                                               const float2* __restrict__ Hb, float2* __restrict__ Cb,
                                               float* __restrict__ Pb, const int* __restrict__ ib, int order) {
    constexpr bool SPLIT = PREC != EELS_FP32;
    static_assert(!(SPLIT && KIND == 1), "the [k][n] B layout is single precision only");
    static_assert(!(SPLIT && EPI == 2), "split Gram tiles run in the SC kernel");
    constexpr int LDS_BYTES = SPLIT ? 4 * BM * LDS_ * 4 : 2 * BM * LDF * 8;
    __shared__ __attribute__((aligned(16))) char smem[LDS_BYTES > 2048 ? LDS_BYTES : 2048];

    // ---- locate this block's problem and tile
    int tm, tn, t;
    const GemmDesc& d = descs[locate_tile(descs, n_desc, order, tm, tn, t, blockIdx.x, gridDim.x)];
    if constexpr (EPI == 2) {
        if (tn < tm) return;   // Gram tiles: the lower triangle is the conjugate transpose
    }
    const int M = d.M, K = d.K, N = d.N_inner;
    const int m0 = tm * BM, n0 = tn * BN;
    const float2* A = Ab + d.a_off + (int64_t)t * d.a_tstride;
    const float2* B = Bb + d.b_off + (int64_t)t * d.b_tstride;
    const float2* Hrow = d.h_off >= 0 && Hb ? Hb + d.h_off + (int64_t)t * d.ldh : nullptr;
    const int* idx = d.idx_off >= 0 ? ib + d.idx_off : nullptr;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int li = lane & 31, hl = lane >> 5;

    // ---- per-thread global load assignment (4 float4 = 8 complex for each operand)
    int64_t a_row[4];
    int b_kc[4];
    int64_t b_row[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        int f = tid + l * 256;
        int row = f >> 3;
        int m = m0 + row;
        a_row[l] = -1;
        if (m < M) a_row[l] = (int64_t)((KIND == 1 && idx) ? idx[m] : m) * d.lda;
        if constexpr (KIND == 0) {
            int n = n0 + row;
            b_row[l] = -1;
            if (n < N) b_row[l] = (int64_t)(idx ? idx[n] : n) * d.ldb;
            b_kc[l] = (f & 7) * 2;
        } else {
            b_kc[l] = f >> 6;           // k row of the [k][n] tile
            b_row[l] = (f & 63) * 2;    // column pair within the tile
        }
    }

    float4 ra[4], rb[4];
    auto gload = [&](int k0) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            int kc = ((tid + l * 256) & 7) * 2;
            int k = k0 + kc;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (a_row[l] >= 0 && k < K) {
                v = *(const float4*)(A + a_row[l] + k);
                if (k + 1 >= K) v.z = v.w = 0.f;
            }
            ra[l] = v;
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (KIND == 0) {
                int k = k0 + b_kc[l];
                if (b_row[l] >= 0 && k < K) {
                    v = *(const float4*)(B + b_row[l] + k);
                    if (k + 1 >= K) v.z = v.w = 0.f;
                    if (Hrow) {
                        float2 h0 = Hrow[k];
                        float2 h1 = k + 1 < K ? Hrow[k + 1] : make_float2(0.f, 0.f);
                        float2 x0 = cmul2(make_float2(v.x, v.y), h0), x1 = cmul2(make_float2(v.z, v.w), h1);
                        v = make_float4(x0.x, x0.y, x1.x, x1.y);
                    }
                }
            } else {
                int k = k0 + b_kc[l];
                int n = n0 + (int)b_row[l];
                if (k < K && n < N) {
                    v = *(const float4*)(B + (int64_t)k * d.ldb + n);
                    if (n + 1 >= N) v.z = v.w = 0.f;
                }
            }
            rb[l] = v;
        }
    };

    auto sstore = [&]() {
        if constexpr (!SPLIT) {
            float2* As = (float2*)smem;
            float2* Bs = As + BM * LDF;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                int f = tid + l * 256;
                int row = f >> 3, kc = (f & 7) * 2;
                As[row * LDF + kc] = make_float2(ra[l].x, ra[l].y);
                As[row * LDF + kc + 1] = make_float2(ra[l].z, ra[l].w);
                if constexpr (KIND == 0) {
                    Bs[row * LDF + kc] = make_float2(rb[l].x, rb[l].y);
                    Bs[row * LDF + kc + 1] = make_float2(rb[l].z, rb[l].w);
                } else {
                    int kr = b_kc[l], nc = (int)b_row[l];
                    Bs[nc * LDF + kr] = make_float2(rb[l].x, rb[l].y);
                    Bs[(nc + 1) * LDF + kr] = make_float2(rb[l].z, rb[l].w);
                }
            }
        } else {
            uint32_t* Ah = (uint32_t*)smem;
            uint32_t* Al = Ah + BM * LDS_;
            uint32_t* Bh = Al + BM * LDS_;
            uint32_t* Bl = Bh + BN * LDS_;
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                int f = tid + l * 256;
                int row = f >> 3, kc = (f & 7) * 2;
                uint32_t h0, l0, h1, l1;
                split2<PREC>(ra[l].x, ra[l].y, h0, l0);
                split2<PREC>(ra[l].z, ra[l].w, h1, l1);
                *(uint2*)&Ah[row * LDS_ + kc] = make_uint2(h0, h1);
                *(uint2*)&Al[row * LDS_ + kc] = make_uint2(l0, l1);
                split2<PREC>(rb[l].x, rb[l].y, h0, l0);
                split2<PREC>(rb[l].z, rb[l].w, h1, l1);
                *(uint2*)&Bh[row * LDS_ + kc] = make_uint2(h0, h1);
                *(uint2*)&Bl[row * LDS_ + kc] = make_uint2(l0, l1);
            }
        }
    };

    floatx16 accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) { accR[a][b][v] = 0.f; accI[a][b][v] = 0.f; }

    const int nk = (K + BK - 1) / BK;
    gload(0);
    for (int kt = 0; kt < nk; ++kt) {
        __syncthreads();
        sstore();
        __syncthreads();
        if (kt + 1 < nk) gload((kt + 1) * BK);
        if constexpr (!SPLIT) {
            const float* Asf = (const float*)smem;
            const float2* Bs = (const float2*)smem + BM * LDF;
#pragma unroll 4
            for (int kk = 0; kk < BK; ++kk) {
                float a[2], br[2], bi[2];
#pragma unroll
                for (int bm = 0; bm < 2; ++bm) a[bm] = Asf[((wm * 64 + bm * 32 + li) * LDF + kk) * 2 + hl];
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    float2 b = Bs[(wn * 64 + bn * 32 + li) * LDF + kk];
                    if constexpr (EPI == 2) {   // conj(a) b
                        br[bn] = hl ? b.y : b.x;
                        bi[bn] = hl ? -b.x : b.y;
                    } else {
                        br[bn] = hl ? -b.y : b.x;
                        bi[bn] = hl ? b.x : b.y;
                    }
                }
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                    for (int bn = 0; bn < 2; ++bn) {
                        accR[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bm], br[bn], accR[bm][bn], 0, 0, 0);
                        accI[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[bm], bi[bn], accI[bm][bn], 0, 0, 0);
                    }
            }
        } else {
            const uint32_t* Ah = (const uint32_t*)smem;
            const uint32_t* Al = Ah + BM * LDS_;
            const uint32_t* Bh = Al + BM * LDS_;
            const uint32_t* Bl = Bh + BN * LDS_;
#pragma unroll
            for (int ks = 0; ks < BK / 8; ++ks) {
                u32x4 ah[2], al[2], brh[2], brl[2], bih[2], bil[2];
#pragma unroll
                for (int bm = 0; bm < 2; ++bm) {
                    int o = (wm * 64 + bm * 32 + li) * LDS_ + ks * 8 + hl * 4;
                    ah[bm] = *(const u32x4*)&Ah[o];
                    al[bm] = *(const u32x4*)&Al[o];
                }
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    int o = (wn * 64 + bn * 32 + li) * LDS_ + ks * 8 + hl * 4;
                    u32x4 bh = *(const u32x4*)&Bh[o];
                    u32x4 bl = *(const u32x4*)&Bl[o];
                    brh[bn] = neg_imag(bh);
                    brl[bn] = neg_imag(bl);
                    bih[bn] = swap_halves(bh);
                    bil[bn] = swap_halves(bl);
                }
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                    for (int bn = 0; bn < 2; ++bn) {
                        accR[bm][bn] = mfma16<PREC>(ah[bm], brh[bn], accR[bm][bn]);
                        accR[bm][bn] = mfma16<PREC>(ah[bm], brl[bn], accR[bm][bn]);
                        accR[bm][bn] = mfma16<PREC>(al[bm], brh[bn], accR[bm][bn]);
                        accI[bm][bn] = mfma16<PREC>(ah[bm], bih[bn], accI[bm][bn]);
                        accI[bm][bn] = mfma16<PREC>(ah[bm], bil[bn], accI[bm][bn]);
                        accI[bm][bn] = mfma16<PREC>(al[bm], bih[bn], accI[bm][bn]);
                    }
            }
        }
    }

    // ---- epilogues.  32x32 accumulator layout: element v of lane l is row
    // 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32.
    if constexpr (EPI == 2) {
        float2* G = (float2*)Pb + d.p_off + (int64_t)t * d.ldc_t;
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int i = n0 + wn * 64 + bn * 32 + li;
            if (i >= N) continue;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    if (m < M) G[(int64_t)m * d.ldc_m + i] = make_float2(accR[bm][bn][v], accI[bm][bn][v]);
                }
        }
    } else if constexpr (EPI == 0) {
        float2* C = Cb + d.c_off + (int64_t)t * d.ldc_t;
        if (d.flags & GD_ZERO_PAD) {
            const int npad = (N + 15) & ~15;
            if (n0 + BN > N && n0 < npad)
                for (int e = tid; e < BM * 16; e += 256) {
                    int m = m0 + e / 16, i = N + e % 16;
                    if (m < M && i < npad && i >= n0 && i < n0 + BN) C[(int64_t)m * d.ldc_m + i] = make_float2(0.f, 0.f);
                }
        }
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int i = n0 + wn * 64 + bn * 32 + li;
            if (i >= N) continue;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    if (m < M) C[(int64_t)m * d.ldc_m + i] = make_float2(accR[bm][bn][v], accI[bm][bn][v]);
                }
        }
    } else {
        __syncthreads();
        float* red = (float*)smem;  // [2][BN]
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            float s = 0.f;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) s += accR[bm][bn][v] * accR[bm][bn][v] + accI[bm][bn][v] * accI[bm][bn][v];
            s += __shfl_xor(s, 32);
            if (hl == 0) red[wm * BN + wn * 64 + bn * 32 + li] = s;
        }
        __syncthreads();
        if (tid < BN) {
            int i = n0 + tid;
            if (i < N) Pb[d.p_off + (int64_t)tm * d.ld_part + (int64_t)t * N + i] = red[tid] + red[BN + tid];
        }
    }
}

// ============================================================================ split GEMM, v2
//
// Split-complex ("SC") storage: a row of Kpad complex values (Kpad % 16 == 0) is Kpad / 4
// units of 32 bytes; unit u holds complex 4u .. 4u+3 as [hi: four u32 (re, im) half pairs]
// [lo: four u32].  Offsets and strides count 8-byte complex slots exactly as for complex64,
// so an SC matrix occupies the same bytes as its complex64 form.
//
// The kernel streams 128-row x BK-complex tiles of both operands (BK = 4 UNITS: 16 or 8)
// straight from global memory into a ring of NSTAGE LDS buffers (global_load_lds_dwordx4,
// no registers), so NSTAGE - 1 tiles are in flight while one is multiplied.  A tile row
// holds QUADS = 2 UNITS 16-byte quads; quad q of row r is stored at position
// q ^ ((r >> 1) & (QUADS - 1)), which makes the fragment reads of consecutive rows hit
// distinct LDS banks.  Two workgroups share a CU when their rings fit in half the LDS
// (16-complex tiles: 2 stages; 8-complex tiles: up to 5 stages).
// Rows beyond M or N are clamped to the last valid row (their results are discarded or
// masked); the K padding of every SC operand holds zeros.


template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    // gfx9 s_waitcnt: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at max
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// WM = 2: 4 waves on a 128 x 128 tile; WM = 4: 8 waves on a 256 x 128 tile (each wave still
// 64 x 64, so its MFMA and LDS work per step is the same, while the block's operand loads per
// flop drop by a quarter; one block per CU)
template <int UNITS, int NSTAGE, int WM>
struct ScPipe {
    static constexpr int ROWB = 32 * UNITS;              // bytes of one tile row
    static constexpr int QUADS = 2 * UNITS;
    static constexpr int BMX = 64 * WM;                  // A rows of the tile
    static constexpr int NW = 2 * WM;                    // waves
    static constexpr int STAGE = (BMX + 128) * ROWB;     // A and B tiles
    static constexpr int RPI = 1024 / ROWB;              // rows per wave-wide 16-byte load
    static constexpr int NIA = 32 / RPI;                 // A loads per wave (32 rows each)
    static constexpr int NIB = 128 / NW / RPI;           // B loads per wave
    static constexpr int WAVES_PER_EU = WM == 2 && 2 * NSTAGE * STAGE <= 160 * 1024 ? 2 : 1;
    static constexpr int G = WM == 2 ? 8 : 4;            // m tiles per group of the XCD-aware order
};

template <int PREC, int EPI, int NSTAGE, int UNITS, int SCHED, int WM>
__global__ __launch_bounds__(128 * WM, (ScPipe<UNITS, NSTAGE, WM>::WAVES_PER_EU)) void k_cgemm_sc(
    const GemmDesc* __restrict__ descs, int n_desc, const uint32_t* __restrict__ Ab, const uint32_t* __restrict__ Bb,
    uint32_t* __restrict__ Cb, float* __restrict__ Pb, const int* __restrict__ ib, int order,
    int* __restrict__ queue, int ntiles, const float2* __restrict__ Hb, float gscale) {
    using SP = ScPipe<UNITS, NSTAGE, WM>;
    constexpr int STAGE = SP::STAGE, ROWB = SP::ROWB, QUADS = SP::QUADS, RPI = SP::RPI, NIA = SP::NIA, NIB = SP::NIB;
    constexpr int BMX = SP::BMX, NT = 128 * WM;
    constexpr int BKS = 4 * UNITS;  // complex per tile row
    static_assert(WM == 2 || EPI != 2, "the 256-row tile has no FP32 Gram-tile epilogue");
    // SCHED bit 2: operands staged through registers (global loads into VGPRs, one tile ahead,
    // written to the LDS stage at the top of the next step) instead of global_load_lds
    constexpr bool REG = (SCHED & 4) != 0;
    static_assert(!REG || NSTAGE == 2, "register staging keeps one tile in flight");
    static_assert(EPI != 4 || NSTAGE * STAGE >= 32 * (BMX + 128) * 8, "the G epilogue stages H in the LDS ring");
    __shared__ __attribute__((aligned(1024))) char smem[NSTAGE * STAGE];
    __shared__ int next_tile;

  // one output tile (bid in 0 .. ntiles-1); a return skips the tile
  auto run_tile = [&](const int bid) {
    int tm, tn, t;
    const GemmDesc& d = descs[locate_tile<SP::G>(descs, n_desc, order, tm, tn, t, bid, ntiles)];
    if constexpr (EPI == 2 || EPI == 4) {
        // Gram tiles: the lower triangle is the conjugate transpose; a tile with no element on
        // or above the diagonal is skipped
        if (tn * BN + BN - 1 < tm * BMX) return;
    }
    const int M = d.M, N = d.N_inner;
    const int m0 = tm * BMX, n0 = tn * BN;
    const int nk = (d.K + BKS - 1) / BKS;
    const char* A = (const char*)Ab + 8 * (d.a_off + (int64_t)t * d.a_tstride);
    const char* B = (const char*)Bb + 8 * (d.b_off + (int64_t)t * d.b_tstride);
    const int* idx = d.idx_off >= 0 ? ib + d.idx_off : nullptr;
    const int* idx_a = (d.flags & GD_IDX_A) ? idx : nullptr;
    const int* idx_b = (d.flags & GD_IDX_A) ? nullptr : idx;

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int li = lane & 31, hl = lane >> 5;

    // this lane's A and B source rows (one per RPI-row chunk of the wave's 32 A rows and
    // 128 / NW B rows)
    constexpr int BRW = 128 / SP::NW;   // B rows loaded per wave
    const int qpos = lane % QUADS;
    const char* asrc[NIA];
    const char* bsrc[NIB];
#pragma unroll
    for (int c = 0; c < NIA; ++c) {
        int r = wave * 32 + c * RPI + lane / QUADS;
        int q = qpos ^ ((r >> 1) & (QUADS - 1));
        int m = min(m0 + r, M - 1);
        int mr = idx_a ? idx_a[m] : m;
        asrc[c] = A + (int64_t)mr * d.lda * 8 + 16 * q;
    }
#pragma unroll
    for (int c = 0; c < NIB; ++c) {
        int r = wave * BRW + c * RPI + lane / QUADS;
        int q = qpos ^ ((r >> 1) & (QUADS - 1));
        int n = min(n0 + r, N - 1);
        int nr = idx_b ? idx_b[n] : n;
        bsrc[c] = B + (int64_t)nr * d.ldb * 8 + 16 * q;
    }
    typedef __attribute__((address_space(3))) char lds_char;
    lds_char* lds = (lds_char*)smem;
    auto issue = [&](int kt) {
        lds_char* st = lds + (kt % NSTAGE) * STAGE;
        int64_t koff = (int64_t)kt * ROWB;
#pragma unroll
        for (int c = 0; c < NIA; ++c)
            __builtin_amdgcn_global_load_lds((const void*)(asrc[c] + koff), (void*)(st + (wave * 32 + c * RPI) * ROWB),
                                             16, 0, 0);
#pragma unroll
        for (int c = 0; c < NIB; ++c)
            __builtin_amdgcn_global_load_lds((const void*)(bsrc[c] + koff),
                                             (void*)(st + BMX * ROWB + (wave * BRW + c * RPI) * ROWB), 16, 0, 0);
    };

    floatx16 accR[2][2], accI[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) { accR[a][b][v] = 0.f; accI[a][b][v] = 0.f; }

    // operand fragments of one 8-complex step: hi and lo quads of this lane's A and B rows
    struct Frag {
        u32x4 ah[2], al[2], bh[2], bl[2];
    };
    auto load_frag = [&](const char* st, int ks, Frag& f) {
        const int u = 2 * ks + hl;
#pragma unroll
        for (int bm = 0; bm < 2; ++bm) {
            int r = wm * 64 + bm * 32 + li;
            int sw = (r >> 1) & (QUADS - 1);
            const char* row = st + r * ROWB;
            f.ah[bm] = *(const u32x4*)(row + 16 * ((2 * u) ^ sw));
            f.al[bm] = *(const u32x4*)(row + 16 * ((2 * u + 1) ^ sw));
        }
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int r = wn * 64 + bn * 32 + li;
            int sw = (r >> 1) & (QUADS - 1);
            const char* row = st + BMX * ROWB + r * ROWB;
            f.bh[bn] = *(const u32x4*)(row + 16 * ((2 * u) ^ sw));
            f.bl[bn] = *(const u32x4*)(row + 16 * ((2 * u + 1) ^ sw));
        }
    };
    auto mma = [&](const Frag& f) {
        if constexpr (SCHED & 2) __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            // Re C = A'.(Br, -Bi), Im C = A'.(Bi, Br); with conj(A) (Gram tiles):
            // Re C = A'.(Br, Bi), Im C = A'.(Bi, -Br)
            u32x4 brh, brl, bih, bil;
            if constexpr (EPI == 2 || EPI == 4) {
                brh = f.bh[bn]; brl = f.bl[bn];
                bih = neg_imag(swap_halves(f.bh[bn])); bil = neg_imag(swap_halves(f.bl[bn]));
            } else {
                brh = neg_imag(f.bh[bn]); brl = neg_imag(f.bl[bn]);
                bih = swap_halves(f.bh[bn]); bil = swap_halves(f.bl[bn]);
            }
#pragma unroll
            for (int bm = 0; bm < 2; ++bm) {
                accR[bm][bn] = mfma16<PREC>(f.ah[bm], brh, accR[bm][bn]);
                accR[bm][bn] = mfma16<PREC>(f.ah[bm], brl, accR[bm][bn]);
                accR[bm][bn] = mfma16<PREC>(f.al[bm], brh, accR[bm][bn]);
                accI[bm][bn] = mfma16<PREC>(f.ah[bm], bih, accI[bm][bn]);
                accI[bm][bn] = mfma16<PREC>(f.ah[bm], bil, accI[bm][bn]);
                accI[bm][bn] = mfma16<PREC>(f.al[bm], bih, accI[bm][bn]);
            }
        }
        if constexpr (SCHED & 2) __builtin_amdgcn_s_setprio(0);
    };

    // register staging: this lane's quads of the next tile, at the LDS positions global_load_lds
    // would give them (lane l of a load writes bytes 16 l .. 16 l + 15 of its rows' block)
    u32x4 stg[REG ? NIA + NIB : 1];
    auto load_stg = [&](int kt) {
        const int64_t koff = (int64_t)kt * ROWB;
#pragma unroll
        for (int c = 0; c < NIA; ++c) stg[c] = *(const u32x4*)(asrc[c] + koff);
#pragma unroll
        for (int c = 0; c < NIB; ++c) stg[NIA + c] = *(const u32x4*)(bsrc[c] + koff);
    };
    if constexpr (REG) {
        if (nk > 0) load_stg(0);
    } else {
#pragma unroll
        for (int s = 0; s < NSTAGE - 1; ++s)
            if (s < nk) issue(s);
    }

    for (int kt = 0; kt < nk; ++kt) {
        if constexpr (REG) {
            // stage kt % 2 was last read in step kt - 2, which every wave finished before the
            // barrier of step kt - 1
            char* stw = smem + (kt % NSTAGE) * STAGE;
#pragma unroll
            for (int c = 0; c < NIA; ++c) *(u32x4*)(stw + (wave * 32 + c * RPI) * ROWB + lane * 16) = stg[c];
#pragma unroll
            for (int c = 0; c < NIB; ++c)
                *(u32x4*)(stw + BMX * ROWB + (wave * BRW + c * RPI) * ROWB + lane * 16) = stg[NIA + c];
            __syncthreads();
            if (kt + 1 < nk) load_stg(kt + 1);
        } else {
            // this wave's loads of tile kt are done once at most the later tiles' loads remain;
            // the barrier then covers every wave's part of the tile and frees the stage that was
            // multiplied in the previous iteration (its LDS reads fed MFMAs, so they completed)
            if (nk - 1 - kt >= NSTAGE - 2) wait_vmcnt<(NIA + NIB) * (NSTAGE - 2)>();
            else wait_vmcnt<0>();
            __builtin_amdgcn_s_barrier();
            if (kt + NSTAGE - 1 < nk) issue(kt + NSTAGE - 1);
        }
        const char* st = smem + (kt % NSTAGE) * STAGE;
        if constexpr (SCHED & 1) {
            // fragments of the next 8-complex step are read while this step's MFMAs run
            Frag f[2];
            load_frag(st, 0, f[0]);
#pragma unroll
            for (int ks = 0; ks < UNITS / 2; ++ks) {
                if (ks + 1 < UNITS / 2) load_frag(st, ks + 1, f[(ks + 1) & 1]);
                mma(f[ks & 1]);
            }
        } else {
#pragma unroll
            for (int ks = 0; ks < UNITS / 2; ++ks) {
                Frag f;
                load_frag(st, ks, f);
                mma(f);
            }
        }
    }

    if constexpr (EPI == 2) {
        float2* G = (float2*)Pb + d.p_off + (int64_t)t * d.ldc_t;
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int i = n0 + wn * 64 + bn * 32 + li;
            if (i >= N) continue;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    if (m < M) G[(int64_t)m * d.ldc_m + i] = make_float2(accR[bm][bn][v], accI[bm][bn][v]);
                }
        }
    } else if constexpr (EPI == 4) {
        // Window-Gram G tile: G = gscale M o S with M this Gram tile and S(m, i) =
        // sum_t conj(H_t[m]) H_t[i] over the site's nt <= 32 transitions (h_off, ldh apart;
        // ld_part holds nt).  G is Hermitian: an element on or above the diagonal (i >= m) is
        // stored SC at [m][i], and one above it also as its conjugate at [i][m], so every element
        // of G is written once; columns N .. ldc_m - 1 of every row are zero.
        __syncthreads();                 // every wave is past its last fragment read: the ring is free
        const int nt = (int)d.ld_part;
        const float2* Hs = Hb + d.h_off;
        float2* hrow = (float2*)smem;    // [t][BMX]: H_t at the tile's rows m0 + x
        float2* hcol = hrow + 32 * BMX;  // [t][128]: H_t at its columns n0 + x
        for (int w = tid; w < nt * BMX; w += NT) {
            const int tt = w / BMX, x = w % BMX;
            hrow[w] = m0 + x < M ? Hs[(int64_t)tt * d.ldh + m0 + x] : make_float2(0.f, 0.f);
        }
        for (int w = tid; w < nt * 128; w += NT) {
            const int tt = w >> 7, x = w & 127;
            hcol[w] = n0 + x < N ? Hs[(int64_t)tt * d.ldh + n0 + x] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const int64_t cbase = d.c_off, ldg = d.ldc_m;
        if (n0 + BN > N && n0 < ldg) {
            for (int e = tid; e < BMX * 16; e += NT) {
                const int m = m0 + e / 16, i = N + e % 16;
                if (m < M && i < ldg && i >= n0 && i < n0 + BN)
                    sc_store(Cb, cbase + (int64_t)m * ldg + i, make_float2(0.f, 0.f), PREC);
            }
        }
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            const int il = wn * 64 + bn * 32 + li, i = n0 + il;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm) {
                const int mb = wm * 64 + bm * 32 + 4 * hl;   // row of v = 0 in the tile
                float sr[16], si[16];
#pragma unroll
                for (int v = 0; v < 16; ++v) { sr[v] = 0.f; si[v] = 0.f; }
                for (int tt = 0; tt < nt; ++tt) {
                    const float2 b = hcol[tt * 128 + il];
#pragma unroll
                    for (int v = 0; v < 16; ++v) {
                        const float2 a = hrow[tt * BMX + mb + 8 * (v >> 2) + (v & 3)];
                        sr[v] += a.x * b.x + a.y * b.y;     // conj(a) b
                        si[v] += a.x * b.y - a.y * b.x;
                    }
                }
                float gr[16], gi[16];
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const float mr = accR[bm][bn][v], mi = accI[bm][bn][v];
                    gr[v] = gscale * (mr * sr[v] - mi * si[v]);
                    gi[v] = gscale * (mr * si[v] + mi * sr[v]);
                }
                if (i >= N) continue;
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int m = m0 + mb + 8 * (v >> 2) + (v & 3);
                    if (m < M && i >= m) sc_store(Cb, cbase + (int64_t)m * ldg + i, make_float2(gr[v], gi[v]), PREC);
                }
#pragma unroll
                for (int g4 = 0; g4 < 4; ++g4) {
                    const int m4 = m0 + mb + 8 * g4;         // four consecutive columns of row i
                    if (i <= m4) continue;                   // none of them below the diagonal
                    if (i > m4 + 3) {                        // all four (and all < i < M)
                        u32x4 hi, lo;
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            uint32_t h, l;
                            split2<PREC>(gr[4 * g4 + e], -gi[4 * g4 + e], h, l);
                            hi[e] = h;
                            lo[e] = l;
                        }
                        uint32_t* o = Cb + ((cbase + (int64_t)i * ldg + m4) >> 2) * 8;
                        *(u32x4*)o = hi;
                        *(u32x4*)(o + 4) = lo;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (m4 + e < i)
                                sc_store(Cb, cbase + (int64_t)i * ldg + m4 + e,
                                         make_float2(gr[4 * g4 + e], -gi[4 * g4 + e]), PREC);
                    }
                }
            }
        }
    } else if constexpr (EPI == 0) {
        // store the product in SC form; the padding columns N .. ceil16(N)-1 get zeros so
        // that the result can be a K operand of the next product
        const int64_t cbase = d.c_off + (int64_t)t * d.ldc_t;
        const int npad = (N + 15) & ~15;
        if (n0 + BN > N && n0 < npad) {
            for (int e = tid; e < BMX * 16; e += NT) {
                int m = m0 + e / 16, i = N + e % 16;
                if (m < M && i < npad && i >= n0 && i < n0 + BN)
                    sc_store(Cb, cbase + (int64_t)m * d.ldc_m + i, make_float2(0.f, 0.f), PREC);
            }
        }
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int i = n0 + wn * 64 + bn * 32 + li;
            if (i >= N) continue;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    if (m < M) sc_store(Cb, cbase + (int64_t)m * d.ldc_m + i, make_float2(accR[bm][bn][v], accI[bm][bn][v]), PREC);
                }
        }
    } else if constexpr (EPI == 3) {
        // store the product as complex64, zeroing the padding columns N .. ceil16(N)-1
        float2* Cf = (float2*)Cb;
        const int64_t cbase = d.c_off + (int64_t)t * d.ldc_t;
        const int npad = (N + 15) & ~15;
        if (n0 + BN > N && n0 < npad) {
            for (int e = tid; e < BMX * 16; e += NT) {
                int m = m0 + e / 16, i = N + e % 16;
                if (m < M && i < npad && i >= n0 && i < n0 + BN) Cf[cbase + (int64_t)m * d.ldc_m + i] = make_float2(0.f, 0.f);
            }
        }
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            int i = n0 + wn * 64 + bn * 32 + li;
            if (i >= N) continue;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    if (m < M) Cf[cbase + (int64_t)m * d.ldc_m + i] = make_float2(accR[bm][bn][v], accI[bm][bn][v]);
                }
        }
    } else {
        __syncthreads();
        float* red = (float*)smem;
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            float s = 0.f;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    int m = m0 + wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * hl + (v & 3);
                    float x = accR[bm][bn][v] * accR[bm][bn][v] + accI[bm][bn][v] * accI[bm][bn][v];
                    s += m < M ? x : 0.f;
                }
            s += __shfl_xor(s, 32);
            if (hl == 0) red[wm * BN + wn * 64 + bn * 32 + li] = s;
        }
        __syncthreads();
        if (tid < BN) {
            int i = n0 + tid;
            float acc = red[tid];
#pragma unroll
            for (int w = 1; w < WM; ++w) acc += red[w * BN + tid];
            if (i < N) Pb[d.p_off + (int64_t)tm * d.ld_part + (int64_t)t * N + i] = acc;
        }
    }
  };

    if (!queue) {
        run_tile(blockIdx.x);
        return;
    }
    // persistent: the resident workgroups take tiles from the work queue until it runs dry
    for (;;) {
        if (threadIdx.x == 0) next_tile = atomicAdd(queue, 1);
        __syncthreads();                 // the previous tile's LDS reads are done, next_tile set
        const int bid = next_tile;
        __syncthreads();                 // every thread has read next_tile
        if (bid >= ntiles) break;
        run_tile(bid);
    }
}


template <int PREC, int KIND, int EPI>
static void go(const GemmDesc* dd, int nd, int tiles, const float2* A, const float2* B, const float2* H, float2* C,
               float* P, const int* idx, hipStream_t st) {
    hipLaunchKernelGGL((k_cgemm<PREC, KIND, EPI>), dim3(tiles), dim3(256), 0, st, dd, nd, A, B, H, C, P, idx,
                       tune_get(TUNE_TILE_ORDER));
}

void launch_cgemm(int precision, int kind, int epi, const GemmDesc* dd, int nd, int tiles, const float2* A,
                  const float2* B, const float2* H, float2* C, float* part, const int* idx, hipStream_t st) {
    if (tiles <= 0 || nd <= 0) return;
    if (kind == 1) {
        if (epi == 0) go<EELS_FP32, 1, 0>(dd, nd, tiles, A, B, H, C, part, idx, st);
        else go<EELS_FP32, 1, 1>(dd, nd, tiles, A, B, H, C, part, idx, st);
        return;
    }
    switch (precision) {
        case EELS_FP32:
            if (epi == 0) go<EELS_FP32, 0, 0>(dd, nd, tiles, A, B, H, C, part, idx, st);
            else if (epi == 2) go<EELS_FP32, 0, 2>(dd, nd, tiles, A, B, H, C, part, idx, st);
            else go<EELS_FP32, 0, 1>(dd, nd, tiles, A, B, H, C, part, idx, st);
            break;
        case EELS_BF16_SPLIT:
            if (epi == 0) go<EELS_BF16_SPLIT, 0, 0>(dd, nd, tiles, A, B, H, C, part, idx, st);
            else go<EELS_BF16_SPLIT, 0, 1>(dd, nd, tiles, A, B, H, C, part, idx, st);
            break;
        default:
            if (epi == 0) go<EELS_FP16_SPLIT, 0, 0>(dd, nd, tiles, A, B, H, C, part, idx, st);
            else go<EELS_FP16_SPLIT, 0, 1>(dd, nd, tiles, A, B, H, C, part, idx, st);
            break;
    }
}


// Workgroups of one kernel that are resident at once on the whole device (persistent grids).
template <typename KERN>
static int resident_blocks(KERN kern, int block) {
    static thread_local int n_cu = 0;
    if (n_cu == 0) {
        int dev = 0;
        hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu <= 0) n_cu = 256;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, 0) != hipSuccess || per <= 0) per = 1;
    return n_cu * per;
}

template <int PREC, int EPI>
static void go_sc(int nstage, int rows, const GemmDesc* dd, int nd, int tiles, const uint32_t* A, const uint32_t* B,
                  uint32_t* C, float* P, const int* idx, hipStream_t st, int* queue, const float2* H, float gscale) {
    // pipeline variants: 2 / 3 stages of 16-complex tiles, 4 / 5 stages of 8-complex tiles;
    // 256-row tiles (store epilogue) with two stages of 16-complex tiles.  With a work queue the
    // grid is the device's resident workgroups, which take the tiles from the queue.
    const int order = queue ? 0 : tune_get(TUNE_TILE_ORDER);
#define SCV(NS, U, SC)                                                                                                 \
    do {                                                                                                               \
        auto kern = k_cgemm_sc<PREC, EPI, NS, U, SC, 2>;                                                               \
        const int grid = queue ? std::min(tiles, resident_blocks(kern, 256)) : tiles;                                  \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), 0, st, dd, nd, A, B, C, P, idx, order, queue, tiles, H,      \
                           gscale);                                                                                    \
    } while (0)
    // register staging of the operands: 256-row tiles with key 11 >= 1, 128-row ones with 2
    const int staging = tune_get(TUNE_GEMM_STAGING);
    if constexpr (EPI != 2) {
        if (rows == 256) {
            // two stages of 16-complex tiles (96 KB of LDS; three stages measured slower on the
            // nanoparticle map's Z product, 2.87 against 2.82 s per map)
#define SC256(SC)                                                                                                      \
    do {                                                                                                               \
        auto kern = k_cgemm_sc<PREC, EPI, 2, 4, SC, 4>;                                                                \
        const int grid = queue ? std::min(tiles, resident_blocks(kern, 512)) : tiles;                                  \
        hipLaunchKernelGGL(kern, dim3(grid), dim3(512), 0, st, dd, nd, A, B, C, P, idx, order, queue, tiles, H,      \
                           gscale);                                                                                    \
    } while (0)
            if (staging >= 1) SC256(4);
            else SC256(0);
#undef SC256
            return;
        }
    }
    switch (nstage) {
        case 3: SCV(3, 4, 0); break;
        case 4: SCV(4, 2, 0); break;
        case 5: SCV(5, 2, 0); break;
        default:
            if (staging == 2) {
                SCV(2, 4, 4);
                break;
            }
            switch (tune_get(TUNE_SC_SCHED)) {
                case 1: SCV(2, 4, 1); break;
                case 2: SCV(2, 4, 2); break;
                case 3: SCV(2, 4, 3); break;
                default: SCV(2, 4, 0); break;
            }
            break;
    }
#undef SCV
}

void launch_cgemm_sc(int precision, int epi, int nstage, const GemmDesc* dd, int nd, int tiles, const void* A,
                     const void* B, void* C, float* part, const int* idx, hipStream_t st, int rows, int* queue,
                     const float2* H, float gscale) {
    if (tiles <= 0 || nd <= 0) return;
    const uint32_t *a = (const uint32_t*)A, *b = (const uint32_t*)B;
    uint32_t* c = (uint32_t*)C;
#define SCE(P_)                                                                                                        \
    do {                                                                                                               \
        if (epi == 0) go_sc<P_, 0>(nstage, rows, dd, nd, tiles, a, b, c, part, idx, st, queue, H, gscale);             \
        else if (epi == 2) go_sc<P_, 2>(nstage, rows, dd, nd, tiles, a, b, c, part, idx, st, queue, H, gscale);        \
        else if (epi == 3) go_sc<P_, 3>(nstage, rows, dd, nd, tiles, a, b, c, part, idx, st, queue, H, gscale);        \
        else if (epi == 4) go_sc<P_, 4>(nstage, rows, dd, nd, tiles, a, b, c, part, idx, st, queue, H, gscale);        \
        else go_sc<P_, 1>(nstage, rows, dd, nd, tiles, a, b, c, part, idx, st, queue, H, gscale);                      \
    } while (0)
    if (precision == EELS_BF16_SPLIT) SCE(EELS_BF16_SPLIT);
    else SCE(EELS_FP16_SPLIT);
#undef SCE
}


}  // namespace eels
