// Raster form of the window-Gram detector sum (the probes on a raster aligned with the beam
// lattice).  For a site with window pixels r and aperture beams k = (f a / L_x, f b / L_y):
//     Psi(R, r) = sum_k c_k(R) S_1[k](r),   Y(R, r) = sum_r' G(r, r') Psi(R, r'),
//     I_site(R) = Re sum_r conj(Psi(R, r)) Y(R, r)
// (the detector sum f^2 sum_{t,q} |A_t(q, R)|^2 of Eq. SHn0 regrouped through the Gram matrix G
// of the site's S_2 window).  With R = R_0 + (i L_x / (f M), j L_y / (f M)) the probe phase
// factors as c_k(R) = c_k(R_0) exp(-2 pi i (a i + b j) / M), so for every window pixel both
// Psi(., r) and Y(., r) (the latter from Z = G S_1w^T) are M x M forward DFTs over the beam
// lattice, evaluated at all residues (i mod M, j mod M) at once.
//
// One block (256 threads) takes a run of a site's window pixels.  Per pixel it loads the two
// grids straight into registers (thread 4 s + t holds grid row s, columns t + 4 m; the beams
// were ordered so that these loads are contiguous; in split precision one pixel ahead), runs the
// row DFTs in registers (fft_reg),
// transposes through LDS, runs the column DFTs, and accumulates Re(conj(Psi) Y) per residue in
// registers.  Two blocks share a CU (two waves per SIMD hide the loads' latency).  The block's M^2 partial sums go to `part`; the
// FP64 reduction adds a probe's residue over the site's blocks.
#include <hip/hip_runtime.h>

#include "fft_reg.h"
#include "internal.h"
#include "kernels.h"
#include "stream_store.h"

namespace eels {

namespace {

// Loads the two grids of window pixel r (thread 4 s + t: row s, columns t + 4 m).
__device__ __forceinline__ void load_grids(float2 (&a)[16], float2 (&b)[16], const float2* __restrict__ xr,
                                           const float2* __restrict__ zr, const int (&q)[16]) {
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        a[m] = q[m] >= 0 ? ld_stream(xr + q[m]) : make_float2(0.f, 0.f);
        b[m] = q[m] >= 0 ? ld_stream(zr + q[m]) : make_float2(0.f, 0.f);
    }
}

// PRE: Xt and Z already hold the factor c_k(R_0) of their beam (the split path folds it into the
// S_1 window transpose and its SC copy), and the registers this frees hold the next pixel's grids,
// loaded while the current pixel is transformed.  Otherwise (FP32) the factors are applied here.
template <int M, bool PRE>
__global__ __launch_bounds__(256) void k_raster_dot(const RasterJob* __restrict__ jobs, const float2* __restrict__ base,
                                                    const float2* __restrict__ c0, const int* __restrict__ perm,
                                                    const int* __restrict__ pos, int K, int ld, int chunk,
                                                    float oscale, const float2* __restrict__ tw,
                                                    float* __restrict__ part) {
    static_assert(M == 64, "256 threads hold a 64 x 64 grid");
    // one grid per transform; row s is both the transpose slot of row s and the exchange space
    // of the 64-point sequence that thread group s owns (rows first, then column s).  Rows are
    // PadLen<64> = 68 slots apart and the exchanges keep element i at i + i / 16 of its row:
    // a quarter-wave (4 rows x 4 threads) then meets 16 distinct 8-byte bank pairs in every
    // exchange and transpose access (with rows 65 slots apart and no padding, 4 lanes met in
    // one bank pair).
    constexpr int LD = PadLen<M>::value;
    __shared__ float2 la[M * LD], lb[M * LD];
    const RasterJob jb = jobs[blockIdx.y];
    const int r0 = blockIdx.x * chunk, r1 = min(K, r0 + chunk);
    const int s = threadIdx.x >> 2, t = threadIdx.x & 3;
    int q[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) q[m] = pos[s * M + t + 4 * m];
    float acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = 0.f;
    const float2* xt = base + jb.xt;
    const float2* z = base + jb.z;
    // PRE: the next pixel's grids; otherwise the beams' factors c_k(R_0)
    float2 na[16], nb[16];
    if constexpr (PRE) {
        if (r0 < r1) load_grids(na, nb, xt + (int64_t)r0 * ld, z + (int64_t)r0 * ld, q);
    } else {
#pragma unroll
        for (int m = 0; m < 16; ++m) na[m] = q[m] >= 0 ? c0[perm[q[m]]] : make_float2(0.f, 0.f);
    }
    for (int r = r0; r < r1; ++r) {
        float2 a[16], b[16];
        if constexpr (PRE) {
#pragma unroll
            for (int m = 0; m < 16; ++m) { a[m] = na[m]; b[m] = nb[m]; }
            if (r + 1 < r1) load_grids(na, nb, xt + (int64_t)(r + 1) * ld, z + (int64_t)(r + 1) * ld, q);
        } else {
            load_grids(a, b, xt + (int64_t)r * ld, z + (int64_t)r * ld, q);
#pragma unroll
            for (int m = 0; m < 16; ++m) { a[m] = cmul(na[m], a[m]); b[m] = cmul(na[m], b[m]); }
        }
        // rows: the sequence of row s lies in the 4 lanes 4 s .. 4 s + 3 of one wavefront, so its
        // exchange through row s of the grid needs wave-level ordering only
        fft_reg<M, -1, true, true>(a, la, s * LD, 1, t, tw);
        fft_reg<M, -1, true, true>(b, lb, s * LD, 1, t, tw);
        lds_sync_wave();
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            la[s * LD + t + 4 * m] = a[m];
            lb[s * LD + t + 4 * m] = b[m];
        }
        __syncthreads();                 // every row transformed and written
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            a[m] = la[(t + 4 * m) * LD + s];
            b[m] = lb[(t + 4 * m) * LD + s];
        }
        __syncthreads();                 // every column read: the rows are free again
        fft_reg<M, -1, true, true>(a, la, s * LD, 1, t, tw);      // column s
        fft_reg<M, -1, true, true>(b, lb, s * LD, 1, t, tw);
#pragma unroll
        for (int m = 0; m < 16; ++m) acc[m] = fmaf(a[m].x, b[m].x, fmaf(a[m].y, b[m].y, acc[m]));
    }
    // thread (column i = s, t) holds the residues (i, j = t + 4 m)
    float* out = part + jb.part + (int64_t)blockIdx.x * M * M;
#pragma unroll
    for (int m = 0; m < 16; ++m) out[s + M * (t + 4 * m)] = oscale * acc[m];
}

}  // namespace

void launch_raster_dot(const RasterJob* jobs, int n_jobs, const float2* base, const float2* c0, const int* perm,
                       const int* pos, int M, int K, int ld, int chunk, float oscale, const float2* tw, float* part,
                       hipStream_t st, bool premultiplied) {
    if (n_jobs <= 0 || K <= 0) return;
    dim3 grid((unsigned)ceil_div(K, chunk), (unsigned)n_jobs);
    if (M != 64) return;
    if (premultiplied)
        hipLaunchKernelGGL((k_raster_dot<64, true>), grid, dim3(256), 0, st, jobs, base, c0, perm, pos, K, ld, chunk,
                           oscale, tw, part);
    else
        hipLaunchKernelGGL((k_raster_dot<64, false>), grid, dim3(256), 0, st, jobs, base, c0, perm, pos, K, ld, chunk,
                           oscale, tw, part);
}

}  // namespace eels
