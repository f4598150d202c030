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
    int ldx;                // row stride of the state (live columns padded to 16)
    const float2* cfac = nullptr;   // per-beam factor folded into the captured values (or none)
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
    int ldx;                // row stride of the scratch rows
};

void launch_twiddles(float2* tw, int n, hipStream_t st);
void launch_transmission(float2* T, const float* V, int64_t n, double sigma, hipStream_t st);
// Propagator factor tables, slice j at P + j (nlx + ny): column factors then row factors.
void launch_propagator(float2* P, const double* dz, const Plan& p, hipStream_t st);
// c_k(R) for the first n_probes probes (-1: all of the plan's), rows of N1pad
void launch_probe_coefficients(void* C, const int4* beams, const double* probes, const Plan& p, int sc,
                               hipStream_t st, int n_probes = -1);
void launch_init_band(void* bcap, int64_t bstride, const int4* beams, const int* band_h, const int* band_off,
                      const Plan& p, int sc, hipStream_t st);
void launch_band_fft(int nx, int ny, const BandFft& a, hipStream_t st);
// Row stage of the band FFT alone: rows of FFT_x(T_j * H_t * W_i) (live columns, rows of
// p.ldx) into out[((t Ni + i) ny + y) ldx]; H planes hstride apart, W planes wstride apart.
void launch_band_rows(float2* out, const float2* W, int64_t wstride, int Ni, int nt, const Plan& p, const float2* Tj,
                      const float2* H, int64_t hstride, const float2* tw, hipStream_t st);
void launch_hmul(void* X, const float2* W, int64_t wstride, const float2* H, int64_t hstride, int Ni, int nt, int K,
                 int ld, int sc, hipStream_t st);
void launch_init_forward(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_init_reverse(float2* S, const int4* beams, const Plan& p, hipStream_t st);
void launch_fill_zero(void* ptr, size_t bytes, hipStream_t st);
void launch_fill_zero_d(double* p, int64_t n, hipStream_t st);
void launch_copy(float2* dst, const float2* src, int64_t n, hipStream_t st);
void launch_row_pass(int nx, int mode, const RowPassArgs& a, hipStream_t st);
// Column pass of slice j: Pj = slice j's propagator tables, band_h = band rows per live column.
void launch_col_pass(int ny, int mode, float2* state, int nbeam, int nlx, int ldx, const float2* Pj, const float2* tw,
                     const int* band_h, const BandCap& bc, hipStream_t st);
void launch_reduce(double* map, int P, const int* rptr, const int* ent, const GemmDesc* descs, const float* part,
                   double scale, hipStream_t st);
void launch_reduce_dense(double* map, int P, const GemmDesc* descs, int d_begin, int d_count, const float* part,
                         double scale, hipStream_t st);

// Grouped complex GEMM (see GemmDesc).  kind 0: B rows are K-contiguous ("NT"); kind 1:
// B is [k][n] ("NN", single precision only).  epi 0: store, epi 1: norm partial sums,
// epi 2: Gram tile conj(A) B^T (upper tiles only) stored as FP32 complex into `part`.
void launch_cgemm(int precision, int kind, int epi, const GemmDesc* d_descs, int n_desc, int total_tiles,
                  const float2* A, const float2* B, const float2* H, float2* C, float* part, const int* idx,
                  hipStream_t st);

// Split-precision grouped GEMM on SC operands (see kernels_gemm.hip); B rows of column
// block t start at b_off + t * ldh.  epi 0 stores C in SC form, epi 1 writes norm partials,
// epi 2 the Gram tile conj(A) B^T as FP32 complex (as launch_cgemm), epi 3 stores C as
// complex64, epi 4 the window-Gram G = gscale (conj(A) B^T) o sum_t conj(H_t) H_t^T in SC,
// both triangles (the descriptor's h_off / ldh locate the site's transition potentials in H,
// ld_part holds their count, at most 32).  The index list gathers B rows, or A rows with
// GD_IDX_A.
// rows: A rows of a tile, 128, or 256 (epi 0 and 3 only; the descriptors' tiles_m must
// count 256-row tiles).
// queue (may be null): a device int, zero before the launch; the grid is then the device's
// resident workgroups, which take tiles from the queue until all total_tiles are done
// (persistent launch, tiles in m-fastest order).
void launch_cgemm_sc(int precision, int epi, int nstage, const GemmDesc* d_descs, int n_desc, int total_tiles,
                     const void* A, const void* B, void* C, float* part, const int* idx, hipStream_t st,
                     int rows = 128, int* queue = nullptr, const float2* H = nullptr, float gscale = 0.f);
// S_1 or S_2 window [n_beams][K] (complex64, rows wstride apart) -> its transpose [K][ldo],
// SC for the split precisions, complex64 for EELS_FP32 (beams n_beams .. ldo-1 zero; ldo a
// multiple of 4, dst 32-byte aligned)
// perm (may be null): output column b takes source row perm[b]
void launch_window_t_sc(void* dst, const float2* src, int64_t wstride, int n_beams, int K, int ldo, int prec,
                        hipStream_t st, const int* perm = nullptr);
// The same three producers over every site of a batch in one launch, the sites' offsets taken
// from the device job table (ProdJob): the window transposes (which 0: the S_2 window s2w ->
// s2t in `prec`; 1: the S_1 window s1w -> xt, rows gathered by perm; 2: the S_1 window s1w ->
// s2t, the first product's operand before the S_2 transpose takes its place), the SC copy of the S_1
// window (s1w -> s1sc) and G (m, h, nt -> g).  Source bases: the S_2 capture or the S_1
// windows; destination base: mid2.  With copy_prec a split precision, the transpose of the S_1
// window (which 1) also writes that window's SC copy [n_beams][copy_ld] (s1sc) from the same
// reads, in place of a separate launch_to_sc_batched.  cph (may be null): every beam b's window
// row is multiplied by cph[b] first (the raster form folds c_k(R_0) into both outputs).
// in_sc: the source windows are stored SC in that split precision (else complex64).
void launch_window_t_batched(void* dst_base, const float2* src_base, const ProdJob* jobs, int n_jobs, int which,
                             int64_t wstride, int n_beams, int K, int ldo, int prec, const int* perm, hipStream_t st,
                             int copy_prec = 0, int copy_ld = 0, const float2* cph = nullptr, int in_sc = 0);
// Zeroes complex slots K .. ld-1 of `rows` SC rows of ld slots (the K padding a split GEMM reads).
void launch_sc_zero_cols(void* base, int64_t rows, int ld, int K, hipStream_t st);
void launch_to_sc_batched(void* dst_base, const float2* src_base, const ProdJob* jobs, int n_jobs, int64_t rows, int K,
                          int ld, int prec, hipStream_t st);
void launch_wgram_combine_batched(void* mid2, const float2* H, const ProdJob* jobs, int n_jobs, int K, int ldm, int ldg,
                                  float gscale, int prec, hipStream_t st);
// Raster form of the window-Gram detector sum (kernels_raster.hip): for each job (site) and
// each block of `chunk` window pixels, the M x M DFTs of c0 o Xt[r] and c0 o Z[r] over the beam
// lattice (column q of a row is grid slot pos^-1(q), beam perm[q]) and part[job.part + block
// M^2 + i + M j] = oscale sum_r Re(conj(Psi) Y) at residue (i, j); Xt and Z rows ld complex.
void launch_raster_dot(const RasterJob* jobs, int n_jobs, const float2* base, const float2* c0, const int* perm,
                       const int* pos, int M, int K, int ld, int chunk, float oscale, const float2* tw, float* part,
                       hipStream_t st, bool premultiplied);
// Window-Gram detector sum: G = gscale M o sum_t conj(H_t) H_t^T as SC rows [K][ldg]
// (complex64 for EELS_FP32) from the FP32 complex Gram tiles M [K][ldm] (upper 128-tiles
// valid); and out[i] = oscale sum_r Re(conj(Psi)Y) over the rows of Psi (SC, complex64 for
// EELS_FP32) and Y (complex64), both ld complex apart.
void launch_wgram_combine(void* G, const float2* M, const float2* H, int nt, int K, int ldm, int ldg, float gscale,
                          int prec, hipStream_t st);
void launch_wgram_dot(float* out, const void* psi, const float2* Y, int rows, int K, int ld, float oscale, int prec,
                      hipStream_t st);
// complex64 [rows][ld] -> SC (columns >= K written as zero)
void launch_to_sc(void* dst, const float2* src, int64_t rows, int K, int ld, int prec, hipStream_t st);
// SC -> complex64 of n contiguous complex slots
void launch_from_sc(float2* dst, const void* src, int64_t n, int prec, hipStream_t st);

// Gram form of the detector sum (kernels_gram.hip).  The upper 128 x 128 tiles of
// G [n1][n1] (FP64 complex) += the sum of `nparts` partials (FP32 complex, [n1][ldp] each,
// part_stride apart; only their upper tiles are read).
void launch_gram_reduce(double* G, const float2* part, int nparts, int64_t part_stride, int n1, int ldp,
                        hipStream_t st);
// dst[b][g] = src[b][g] where mask[g] has `bit`, else 0 (rows of ld complex, n_rows rows).
void launch_mask_band(float2* dst, const float2* src, int n_rows, int ld, const int* mask, int bit, hipStream_t st);
// Fills the lower tiles of G from the upper ones (Hermitian), then map[R] += scale *
// Re(c(R)^H G c(R)) for the P probes; C complex64 [P][ldc]; qpart holds P * ceil(n1 / 64)
// doubles of partial sums (summed in a fixed order).
void launch_quadform(double* map, int P, double* G, int n1, const float2* C, int ldc, double* qpart,
                     double scale, hipStream_t st);

// Conventional multislice (kernels_conv.hip).  Elastic waves of probes p0 .. p0+Ni-1 at the
// entrance of slice 0 in the hybrid layout; col_ptr / col_beam group the aperture beams by
// live column.
void launch_conv_init(float2* state, int Ni, int p0, const Plan& p, const int* col_ptr, const int* col_beam,
                      const int4* beams, const double* probes, hipStream_t st);
// Full-plane copies of windowed transition potentials (org: int4 per plane, see Plan).
void launch_conv_scatter_h(float2* Hfull, const float2* H, const int* org, int n_planes, const Plan& p,
                           hipStream_t st);
// wnorm[w] = sum over band slots g < Kb with mask[g] of |exit[w * stride + g]|^2 (FP64).
void launch_conv_norm(double* wnorm, const float2* exit_band, int64_t stride, int Kb, const int* mask, int64_t n_waves,
                      hipStream_t st);
// map[i] = sum over k < n_k of wnorm[k Ni + i].
void launch_conv_map(double* map, const double* wnorm, int Ni, int64_t n_k, hipStream_t st);

}  // namespace eels
