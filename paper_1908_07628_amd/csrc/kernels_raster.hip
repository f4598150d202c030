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
// were ordered so that these loads are contiguous), runs the row DFTs in registers
// (fft_reg), transposes through LDS, runs the column DFTs, and accumulates
// Re(conj(Psi) Y) per residue in registers.  The block's M^2 partial sums go to `part`; the
// FP64 reduction adds a probe's residue over the site's blocks.
#include <hip/hip_runtime.h>

#include "fft_reg.h"
#include "internal.h"
#include "kernels.h"

namespace eels {

namespace {

template <int M>
__device__ __forceinline__ void dft2d(float2 (&v)[16], float2* lds, int s, int t, const float2* __restrict__ tw) {
    constexpr int LD = M + 1;
    fft_reg<M, -1>(v, lds, s * LD, 1, t, tw);        // row s: on exit v[m] = frequency t + 4 m
    __syncthreads();                                  // the rows' exchange reads are done
#pragma unroll
    for (int m = 0; m < 16; ++m) lds[s * LD + t + 4 * m] = v[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; ++m) v[m] = lds[(t + 4 * m) * LD + s];
    fft_reg<M, -1>(v, lds, s * LD, 1, t, tw);        // column s (its first barrier orders the reads above)
}

template <int M>
__global__ __launch_bounds__(256) void k_raster_dot(const RasterJob* __restrict__ jobs, const float2* __restrict__ base,
                                                    const float2* __restrict__ c0, const int* __restrict__ perm,
                                                    const int* __restrict__ pos, int K, int ld, int chunk,
                                                    float oscale, const float2* __restrict__ tw,
                                                    float* __restrict__ part) {
    static_assert(M == 64, "256 threads hold a 64 x 64 grid");
    __shared__ float2 lds[M * (M + 1)];
    const RasterJob jb = jobs[blockIdx.y];
    const int r0 = blockIdx.x * chunk, r1 = min(K, r0 + chunk);
    const int s = threadIdx.x >> 2, t = threadIdx.x & 3;
    int q[16];
    float2 w[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        q[m] = pos[s * M + t + 4 * m];
        w[m] = q[m] >= 0 ? c0[perm[q[m]]] : make_float2(0.f, 0.f);
    }
    float acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = 0.f;
    const float2* xt = base + jb.xt;
    const float2* z = base + jb.z;
    for (int r = r0; r < r1; ++r) {
        float2 a[16], b[16];
        const float2* xr = xt + (int64_t)r * ld;
        const float2* zr = z + (int64_t)r * ld;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            a[m] = q[m] >= 0 ? cmul(w[m], xr[q[m]]) : make_float2(0.f, 0.f);
            b[m] = q[m] >= 0 ? cmul(w[m], zr[q[m]]) : make_float2(0.f, 0.f);
        }
        dft2d<M>(a, lds, s, t, tw);
        dft2d<M>(b, lds, s, t, tw);
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
                       hipStream_t st) {
    if (n_jobs <= 0 || K <= 0) return;
    dim3 grid((unsigned)ceil_div(K, chunk), (unsigned)n_jobs);
    if (M == 64)
        hipLaunchKernelGGL(k_raster_dot<64>, grid, dim3(256), 0, st, jobs, base, c0, perm, pos, K, ld, chunk, oscale,
                           tw, part);
}

}  // namespace eels
