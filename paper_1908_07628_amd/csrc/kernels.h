// Launchers of the device kernels (all enqueue on the given stream).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace eels {

struct RowPassArgs {
    float2* state;
    int nbeam, ny, nlx, hlx;
    const float2* Tj;
    const float2* tw;
    const int* cap_ptr;     // null: no capture in this pass
    const int* cap_rec;
    void* win;
    int64_t win_beams;      // beams per window (N_1 or N_2)
    int Kpad;
    int sc;                 // capture format: 0 complex64, else the split precision
};

// Band capture of the transposed column pass (after the P multiply): beam b's band
// coefficients go to dst[b * stride + g].  dst == null: no capture.
struct BandCap {
    const int* band_h = nullptr;
    const int* band_off = nullptr;
    void* dst = nullptr;
    int64_t stride = 0;
    int sc = 0;
};

// Band FFT of T_j * H_t * W_i for all (t, i): dst[(t Ni + i) * dstride + g].
struct BandFft {
    void* dst;
    int64_t dstride;
    int Kb;
    const float2* W;
    int64_t wstride;
    int Ni, nt, ny, nlx, hlx;
    const float2* Tj;
    const float2* H;
    int64_t hstride;
    const float2 *twx, *twy;
    const int *band_h, *band_off;
    float2* scratch;
    int sc;
};

void launch_twiddles(float2* tw, int n, hipStream_t st);
void launch_transmission(float2* T, const float* V, int64_t n, double sigma, hipStream_t st);
void launch_propagator(float2* P, const double* dz, const int* band_h, const Plan& p, hipStream_t st);
void launch_probe_coefficients(void* C, const int4* beams, const double* probes, const Plan& p, int sc,
                               hipStream_t st);
void launch_init_band(void* bcap, int64_t bstride, const int4* beams, const int* band_h, const int* band_off,
                      const Plan& p, int sc, hipStream_t st);
void launch_band_fft(int nx, int ny, const BandFft& a, hipStream_t st);
void launch_hmul(void* X, const float2* W, int64_t wstride, const float2* H, int64_t hstride, int Ni, int nt, int K,
                 int ld, int sc, hipStream_t st);
void launch_init_forward(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_init_reverse(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t st);
void launch_fill_zero_d(double* p, int64_t n, hipStream_t st);
void launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t st);
void launch_row_pass(int nx, int mode, const RowPassArgs& a, hipStream_t st);
void launch_col_pass(int ny, int mode, float2* state, int nbeam, int nlx, const float2* Pj, const float2* tw,
                     const BandCap& bc, hipStream_t st);
void launch_reduce(double* map, int P, const int* rptr, const int* ent, const GemmDesc* descs, const float* part,
                   double scale, hipStream_t st);
void launch_reduce_dense(double* map, int P, const GemmDesc* descs, int d_begin, int d_count, const float* part,
                         double scale, hipStream_t st);

// Grouped complex GEMM (see GemmDesc).  kind 0: B rows are K-contiguous ("NT"); kind 1:
// B is [k][n] ("NN", single precision only).  epi 0: store, epi 1: norm partial sums.
void launch_cgemm(int precision, int kind, int epi, const GemmDesc* d_descs, int n_desc, int total_tiles,
                  const float2* A, const float2* B, const float2* H, float2* C, float* part, const int* idx,
                  hipStream_t st);

// Split-precision grouped GEMM on SC operands (see kernels_gemm.hip); B rows of column
// block t start at b_off + t * ldh.  epi 0 stores C in SC form, epi 1 writes norm partials.
void launch_cgemm_sc(int precision, int epi, int nstage, const GemmDesc* d_descs, int n_desc, int total_tiles,
                     const void* A, const void* B, void* C, float* part, const int* idx, hipStream_t st);
// complex64 [rows][ld] -> SC (columns >= K written as zero)
void launch_to_sc(void* dst, const float2* src, int64_t rows, int K, int ld, int prec, hipStream_t st);
// SC -> complex64 of n contiguous complex slots
void launch_from_sc(float2* dst, const void* src, int64_t n, int prec, hipStream_t st);

}  // namespace eels
