// Conventional multislice STEM-EELS (Sec. 3, first algorithm): the kernels that the
// scattering-matrix path does not already have.  Waves use the sweeps' hybrid (kx, y)
// layout: rows of ldx complex holding the live kx columns, one plane of ny rows per wave.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kernels.h"

namespace eels {

namespace {

__device__ __forceinline__ int phys_of_live(int c, int nlx, int ldx) {
    if (nlx == ldx) return c;
    return c <= (nlx - 1) / 2 ? c : c + (ldx - nlx);
}

// Elastic wave of probe R_{p0+i} at the entrance of slice 0 (Eq. illum): psi_hat(k) = c_k(R)
// on the aperture beams.  Its hybrid form in live column c is
//   h(c, y) = sum over the beams k of column c of c_k(R) exp(2 pi i k_y y / ny)
// (an unnormalised inverse FFT along y).  The phase of each term is reduced to a fraction
// of a cycle in double before one sincos.
__global__ void k_conv_init(float2* __restrict__ state, int Ni, int p0, int ny, int nlx, int ldx,
                            const int* __restrict__ col_ptr, const int* __restrict__ col_beam,
                            const int4* __restrict__ beams, const double* __restrict__ probes, double lx, double ly,
                            double lam, double defocus, double cs, double scale) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t total = (int64_t)Ni * ny * nlx;
    if (g >= total) return;
    const int c = (int)(g % nlx);
    const int y = (int)((g / nlx) % ny);
    const int i = (int)(g / ((int64_t)nlx * ny));
    const double rx = probes[2 * (p0 + i)], ry = probes[2 * (p0 + i) + 1];
    double re = 0.0, im = 0.0;
    for (int e = col_ptr[c]; e < col_ptr[c + 1]; ++e) {
        const int4 bm = beams[col_beam[e]];
        const double kx = (double)bm.z / lx, ky = (double)bm.w / ly;
        const double k2 = kx * kx + ky * ky;
        const double chi = M_PI * lam * k2 * (0.5 * cs * lam * lam * k2 - defocus);   // radians
        double u = kx * rx + ky * ry - (double)(((int64_t)bm.y * y) % ny) / (double)ny;  // cycles
        u -= floor(u);
        double s, co;
        sincos(-2.0 * M_PI * u - chi, &s, &co);
        re += co;
        im += s;
    }
    state[((int64_t)i * ny + y) * ldx + phys_of_live(c, nlx, ldx)] =
        make_float2((float)(re * scale), (float)(im * scale));
}

// Full-plane transition potentials of windowed sites: plane r holds H row org[r].x placed
// with its window's corner at (org[r].y, org[r].z) (periodic), zero elsewhere.
__global__ void k_conv_scatter_h(float2* __restrict__ Hfull, const float2* __restrict__ H, const int4* __restrict__ org,
                                 int n_planes, int nx, int ny, int nwx, int nwy) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)n_planes * nx * ny) return;
    const int x = (int)(g % nx);
    const int y = (int)((g / nx) % ny);
    const int r = (int)(g / ((int64_t)nx * ny));
    const int4 o = org[r];
    int dx = x - o.y, dy = y - o.z;
    if (dx < 0) dx += nx;
    if (dy < 0) dy += ny;
    float2 v = make_float2(0.f, 0.f);
    if (dx < nwx && dy < nwy) v = H[((int64_t)o.x * nwy + dy) * nwx + dx];
    Hfull[g] = v;
}

// Detector intensity of each exit wave: sum over its band slots g < Kb with mask[g] of
// |phi_hat(g)|^2, in FP64 with a fixed-order block reduction (one block per wave).
__global__ __launch_bounds__(256) void k_conv_norm(double* __restrict__ wnorm, const float2* __restrict__ exit_band,
                                                   int64_t stride, int Kb, const int* __restrict__ mask) {
    __shared__ double red[256];
    const int64_t w = blockIdx.x;
    const float2* v = exit_band + w * stride;
    double acc = 0.0;
    for (int g = threadIdx.x; g < Kb; g += 256) {
        if (mask[g]) {
            float2 a = v[g];
            acc += (double)a.x * a.x + (double)a.y * a.y;
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) wnorm[w] = red[0];
}

// map[i] = sum over k of wnorm[k Ni + i] (wave k Ni + i belongs to probe i), in order of k.
__global__ void k_conv_map(double* __restrict__ map, const double* __restrict__ wnorm, int Ni, int64_t n_k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Ni) return;
    double s = 0.0;
    for (int64_t k = 0; k < n_k; ++k) s += wnorm[k * Ni + i];
    map[i] = s;
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

void launch_conv_init(float2* state, int Ni, int p0, const Plan& p, const int* col_ptr, const int* col_beam,
                      const int4* beams, const double* probes, hipStream_t st) {
    int64_t n = (int64_t)Ni * p.ny * p.nlx;
    if (n <= 0) return;
    const double scale = 1.0 / std::sqrt((double)p.N1fine);
    hipLaunchKernelGGL(k_conv_init, dim3(blocks_for(n, 256)), dim3(256), 0, st, state, Ni, p0, p.ny, p.nlx, p.ldx,
                       col_ptr, col_beam, beams, probes, p.lx, p.ly, p.lam, p.defocus, p.cs, scale);
}

void launch_conv_scatter_h(float2* Hfull, const float2* H, const int* org, int n_planes, const Plan& p,
                           hipStream_t st) {
    int64_t n = (int64_t)n_planes * p.nx * p.ny;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_conv_scatter_h, dim3(blocks_for(n, 256)), dim3(256), 0, st, Hfull, H, (const int4*)org,
                       n_planes, p.nx, p.ny, p.nwx, p.nwy);
}

void launch_conv_norm(double* wnorm, const float2* exit_band, int64_t stride, int Kb, const int* mask, int64_t n_waves,
                      hipStream_t st) {
    if (n_waves <= 0) return;
    hipLaunchKernelGGL(k_conv_norm, dim3((unsigned)n_waves), dim3(256), 0, st, wnorm, exit_band, stride, Kb, mask);
}

void launch_conv_map(double* map, const double* wnorm, int Ni, int64_t n_k, hipStream_t st) {
    if (Ni <= 0) return;
    hipLaunchKernelGGL(k_conv_map, dim3(blocks_for(Ni, 256)), dim3(256), 0, st, map, wnorm, Ni, n_k);
}

}  // namespace eels
