// Gram form of the detector sum (Eq. TPRISM2 with every probe covering every site).
//
// For one ionised site and transition n the map term is sum_q |sum_k Z_n(q, k) c_k(R)|^2
// = c(R)^H (Z_n^H Z_n) c(R), so the whole map is I(R) = scale * c(R)^H G c(R) with
// G = sum over sites, transitions and slices of Z^H Z.  The contraction GEMM writes the
// upper 128 x 128 tiles of each site's Z^H Z (FP32 accumulation over that site's
// transitions and detector beams); these kernels add them into G in FP64 in a fixed order
// and evaluate the quadratic forms at the end.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"
#include "kernels.h"

namespace eels {

// Upper 128 x 128 tiles of G += the nparts partials (fixed order, FP64).
__global__ void k_gram_reduce(double2* __restrict__ G, const float2* __restrict__ part, int nparts,
                              int64_t part_stride, int n1, int ldp) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n1 * n1) return;
    const int k = (int)(idx / n1), k2 = (int)(idx % n1);
    if (k / GEMM_BM > k2 / GEMM_BN) return;
    const int64_t o = (int64_t)k * ldp + k2;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < nparts; ++s) {
        float2 v = part[s * part_stride + o];
        re += v.x;
        im += v.y;
    }
    double2 g = G[idx];
    g.x += re;
    g.y += im;
    G[idx] = g;
}

// Lower tiles of G from the upper ones: G[k][k'] = conj(G[k'][k]).
__global__ void k_gram_mirror(double2* __restrict__ G, int n1) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n1 * n1) return;
    const int k = (int)(idx / n1), k2 = (int)(idx % n1);
    if (k / GEMM_BM <= k2 / GEMM_BN) return;
    double2 g = G[(int64_t)k2 * n1 + k];
    G[idx] = make_double2(g.x, -g.y);
}

// Block: 64 probes x 64 rows k of v(R, k) = sum_k' G[k][k'] c_k'(R), 256 threads, each
// 4 probes (ty + 16 i) x 4 rows (tx + 16 j); k' advances 16 at a time through LDS.  The
// epilogue forms sum_k Re(conj(c_k(R)) v(R, k)) over the block's rows.
__global__ __launch_bounds__(256) void k_quadform(double* __restrict__ qpart, int P, const double2* __restrict__ G,
                                                  int n1, const float2* __restrict__ C, int ldc) {
    __shared__ double2 cs[64][17];
    __shared__ double2 gs[64][17];
    const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
    const int r0 = blockIdx.x * 64, k0 = blockIdx.y * 64;
    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
    for (int kb = 0; kb < n1; kb += 16) {
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const int e = tid + 256 * l, row = e >> 4, col = e & 15;
            const int kk = kb + col;
            const int R = r0 + row, k = k0 + row;
            double2 cv = make_double2(0.0, 0.0), gv = make_double2(0.0, 0.0);
            if (R < P && kk < n1) {
                float2 c = C[(int64_t)R * ldc + kk];
                cv = make_double2(c.x, c.y);
            }
            if (k < n1 && kk < n1) gv = G[(int64_t)k * n1 + kk];
            cs[row][col] = cv;
            gs[row][col] = gv;
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            double2 c[4], g[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] = cs[ty + 16 * i][kk];
#pragma unroll
            for (int j = 0; j < 4; ++j) g[j] = gs[tx + 16 * j][kk];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc[i][j].x += g[j].x * c[i].x - g[j].y * c[i].y;
                    acc[i][j].y += g[j].x * c[i].y + g[j].y * c[i].x;
                }
        }
        __syncthreads();
    }
    // sum_k Re(conj(c_k) v_k) over this thread's rows, then over the 16 threads of a probe
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int R = r0 + ty + 16 * i;
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + tx + 16 * j;
            if (R < P && k < n1) {
                float2 c = C[(int64_t)R * ldc + k];
                s += (double)c.x * acc[i][j].x + (double)c.y * acc[i][j].y;
            }
        }
#pragma unroll
        for (int off = 8; off >= 1; off >>= 1) s += __shfl_xor(s, off, 16);
        if (tx == 0 && R < P) qpart[(int64_t)blockIdx.y * P + R] = s;
    }
}

__global__ void k_quadform_finish(double* __restrict__ map, int P, const double* __restrict__ qpart, int nkb,
                                  double scale) {
    const int R = blockIdx.x * blockDim.x + threadIdx.x;
    if (R >= P) return;
    double s = 0.0;
    for (int b = 0; b < nkb; ++b) s += qpart[(int64_t)b * P + R];
    map[R] += scale * s;
}

__global__ void k_mask_band(float2* __restrict__ dst, const float2* __restrict__ src, int64_t n, int ld,
                            const int* __restrict__ mask, int bit) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dst[i] = (mask[i % ld] & bit) ? src[i] : make_float2(0.f, 0.f);
}

void launch_mask_band(float2* dst, const float2* src, int n_rows, int ld, const int* mask, int bit, hipStream_t st) {
    const int64_t n = (int64_t)n_rows * ld;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mask_band, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n, ld, mask, bit);
}

void launch_gram_reduce(double* G, const float2* part, int nparts, int64_t part_stride, int n1, int ldp,
                        hipStream_t st) {
    const int64_t n = (int64_t)n1 * n1;
    if (n <= 0 || nparts <= 0) return;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (double2*)G, part,
                       nparts, part_stride, n1, ldp);
}

void launch_quadform(double* map, int P, double* G, int n1, const float2* C, int ldc, double* qpart,
                     double scale, hipStream_t st) {
    if (P <= 0 || n1 <= 0) return;
    const int nkb = (n1 + 63) / 64;
    const int64_t n = (int64_t)n1 * n1;
    hipLaunchKernelGGL(k_gram_mirror, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (double2*)G,
                       n1);
    hipLaunchKernelGGL(k_quadform, dim3((unsigned)((P + 63) / 64), (unsigned)nkb), dim3(256), 0, st, qpart, P,
                       (const double2*)G, n1, C, ldc);
    hipLaunchKernelGGL(k_quadform_finish, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, map, P, qpart, nkb,
                       scale);
}

}  // namespace eels
