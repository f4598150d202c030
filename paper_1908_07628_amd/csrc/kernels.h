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
    float2* win;
    int64_t win_beams;      // beams per window (N_1 or N_2)
    int Kpad;
};

void launch_twiddles(float2* tw, int n, hipStream_t st);
void launch_transmission(float2* T, const float* V, int64_t n, double sigma, hipStream_t st);
void launch_propagator(float2* P, const double* dz, const Plan& p, hipStream_t st);
void launch_probe_coefficients(float2* C, const int4* beams, const double* probes, const Plan& p, hipStream_t st);
void launch_init_forward(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_init_reverse(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t st);
void launch_fill_zero_d(double* p, int64_t n, hipStream_t st);
void launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t st);
void launch_row_pass(int nx, int mode, const RowPassArgs& a, hipStream_t st);
void launch_col_pass(int ny, int mode, float2* state, int nbeam, int nlx, const float2* Pj, const float2* tw,
                     hipStream_t st);
void launch_reduce(double* map, int P, const int* rptr, const int* ent, const GemmDesc* descs, const float* part,
                   double scale, hipStream_t st);
void launch_reduce_dense(double* map, int P, const GemmDesc* descs, int d_begin, int d_count, const float* part,
                         double scale, hipStream_t st);

// Grouped complex GEMM (see GemmDesc).  kind 0: B rows are K-contiguous ("NT"); kind 1:
// B is [k][n] ("NN", single precision only).  epi 0: store, epi 1: norm partial sums.
void launch_cgemm(int precision, int kind, int epi, const GemmDesc* d_descs, int n_desc, int total_tiles,
                  const float2* A, const float2* B, const float2* H, float2* C, float* part, const int* idx,
                  hipStream_t st);

}  // namespace eels
