// Internal declarations shared by the host planner and the device orchestration.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "eels.h"

namespace eels {

// Thread-local error text behind eels_last_error().
void set_error(const std::string& msg);

// One capture record: copy pixels x0 .. x0+nwx-1 (mod nx) of a real-space row into
// row `dy` of window `win` (window-local pixel index dy*nwx + u).
struct CaptureRec {
    int win, dy, x0, nwx;
};

// One complex-GEMM problem of a grouped launch.  All offsets count elements of the
// base buffers given at launch time (complex elements for A/B/H/C, floats for the
// partial sums, ints for the index lists).  The output has n_t column blocks of
// N_inner columns; for block t:
//   C_t[m][i] = sum_k A_t[m][k] * B_t[i][k],   A_t = A + t*a_tstride,
//   B_t[i][k] = Bsrc_t[idx ? idx[i] : i][k] * (H ? H[t*ldh + k] : 1),  Bsrc_t = B + t*b_tstride.
// Store epilogue: C[c_off + t*ldc_t + m*ldc_m + i].  Norm epilogue:
// part[p_off + mt*ld_part + t*N_inner + i] = sum over the rows m of tile mt of |C_t[m][i]|^2.
// Tiles: tiles_m x tiles_n x n_t (m fastest), tiles_n = ceil(N_inner / 128).
struct GemmDesc {
    int64_t a_off, b_off, h_off, c_off, p_off;
    int64_t lda, ldb, ldh, ldc_m, ldc_t, ld_part, a_tstride, b_tstride;
    int M, N_inner, n_t, K;
    int64_t idx_off;   // offset into the int table, -1 = no gather
    int tiles_m, tiles_n, tile_start;
    int flags;         // GD_* bits
};
// descriptor flags: GD_ZERO_PAD: the plain FP32 store epilogue also zeroes the padding
// columns N .. ceil16(N)-1 of every stored row (they are K padding of a later product);
// GD_IDX_A: the split kernel gathers the A rows through idx (instead of the B rows)
enum { GD_ZERO_PAD = 1, GD_IDX_A = 2 };
static_assert(sizeof(GemmDesc) == 144, "GemmDesc layout");

// Process-wide tuning knobs (set by eels_tune_set; read at launch time).
enum TuneKey {
    TUNE_SC_STAGES = 0, TUNE_TILE_ORDER = 1, TUNE_SC_SCHED = 2, TUNE_GRAM_STACK = 3, TUNE_GEMM1_ROWS = 4,
    TUNE_GEMM2_ROWS = 5, TUNE_WINDOW_GRAM = 6, TUNE_RASTER = 7, TUNE_CHECKPOINT = 8, TUNE_WG_FUSED = 9,
    TUNE_GRAM_ROWS = 10, TUNE_GEMM_STAGING = 11, TUNE_COUNT = 12
};
int tune_get(int key);

struct Batch {
    int slice;
    int order;
    int d1_begin, d1_count, d1_tiles;   // first GEMM (store epilogue)
    int d1_rows = 128;                  // A rows per tile of the first GEMM (128 or 256)
    int d2_begin, d2_count, d2_tiles;   // second GEMM (norm epilogue)
    int d2_rows = 128;                  // A rows per tile of the second GEMM (split norm epilogue: 128 or 256)
    int job_begin, job_count;           // producer jobs run between the two GEMMs (order P) or before
    int64_t red_ptr;                    // int offset of the per-probe CSR row pointers [P+1], -1: dense
    int64_t red_ent;                    // int offset of the CSR entries (pairs: desc, column)
    int64_t n_entries;
    int n_parts;                        // Gram form: FP32 partials of Z^H Z written by the second GEMM
    // window-Gram form (order P, cropped windows): per site the Gram GEMM of the S_2
    // window (dm) and the product of G with Psi (dy); the d2 range then only drives the reduction
    int dm_begin = 0, dm_count = 0, dm_tiles = 0, dm_rows = 128;
    int dy_begin = 0, dy_count = 0, dy_tiles = 0, dy_rows = 128;
    int64_t r_jobs = -1;                // raster form: int offset of the batch's RasterJob table
    int64_t p_jobs = -1;                // window-Gram form: int offset of the batch's ProdJob table
};

// Window-Gram producers of one site, for the batched launches (complex offsets: s2w in the S_2
// capture, s1w in the S_1 windows, h in the transition potentials, the rest in mid2).
struct ProdJob {
    int64_t s2w, s2t, s1w, xt, s1sc, m, g, h;
    int32_t nt, pad;
};
static_assert(sizeof(ProdJob) == 72, "ProdJob layout");

// Raster form of the window-Gram detector sum, per site: complex offsets (in mid2) of the
// site's S_1 window transposed into beam-slot order Xt [K][N1pad] and of Z = G S_1w^T
// [K][N1pad]; the float offset of its DFT-block partial sums in part.
struct RasterJob {
    int64_t xt, z, part;
};
static_assert(sizeof(RasterJob) == 24, "RasterJob layout");

// Producer job: write the H-multiplied operand of one site into mid2, either in the band
// basis (fft2 of T_j H_t W_i) or pixel-wise (H_t W_i), from S_1 windows or from Psi.
struct Job {
    int from_mid;       // 0: W = S_1 window buffer, 1: W = mid (Psi), 2: W = the S_2 window buffer
    int64_t w_off;      // complex offset of the site's first W row
    int64_t win_off;    // complex offset of the site's S_1 window (order P, split: transposed first)
    int Ni, nt;
    int64_t h_off;      // complex offset of the site's first transition potential
    int64_t dst_off;    // complex offset in mid2
    // window-Gram form: complex offsets in mid2 of the site's S_2 window transpose [K][N_2p],
    // the FP32 complex Gram tiles M [K][Kpad], G [K][Kpad] and Y^T [P_s][Kpad]; Psi in mid;
    // the site's first float in part; eligible probes P_s
    int64_t s2t_off = 0, m_off = 0, g_off = 0, y_off = 0, psi_off = 0, part_off = 0;
    int ps = 0;
    // raster form: Xt (complex64, beam-slot order) and the split copy of the S_1 window [N_1][Kpad]
    // (the Z GEMM's B operand); Z sits at y_off
    int64_t xt_off = 0, s1sc_off = 0;
};

struct SliceInfo {
    bool ion = false;
    int group = -1;
    int64_t cap1_ptr = -1, cap1_rec = -1;  // int offsets of the S_1 capture CSR (rows, records)
    int64_t cap2_ptr = -1, cap2_rec = -1;  // same for S_2
    int ckpt_save = -1;                   // S_1 checkpoint slot saved at this slice's entrance
    std::vector<int> batches;
};

struct Group {
    int j_lo, j_hi;                       // ionised slices j_lo..j_hi (inclusive) are captured
    int n_windows;
    int ckpt = -1;                        // checkpoint slot holding S_1 at the entrance of j_lo
};

struct Plan {
    // problem (owned copies)
    int nx, ny;
    double lx, ly;
    int nz;
    std::vector<double> dz;
    double energy, lam, sigma;
    double alpha, beta_in, beta_out, defocus, cs;
    int f;
    double bandlimit, window_A;
    int P;
    std::vector<double> probes;   // [P][2]
    std::vector<eels_site> sites;
    int64_t n_trans_total;
    int precision;
    int order;

    // derived
    double kmax;
    int hlx, nlx;                 // live kx columns: |kx index| <= hlx, count 2*hlx+1
    int ldx;                      // row stride of the sweep state and band scratch (nlx rounded up to 16)
    std::vector<int> ab1, ab2;    // lattice coordinates (a, b) of beams
    int N1, N2, N1fine, N1pad;
    bool full_window;
    bool resident;                // every ionised slice keeps its own S_2 capture
    std::vector<int64_t> slice_w2;  // complex offset of slice j's S_2 capture in the w2 buffer
    bool recip;                   // band-basis contraction (full-cell windows)
    int hwx, hwy, nwx, nwy, K, Kpad;
    std::vector<int> band_h, band_off;          // band rows per live column, band slot offsets
    int Kb, Kbpad;                              // band pixels, padded stride
    int c_sc, w2_sc, mid2_sc;                   // storage formats (0 complex64, else split precision)
    bool gram;                                  // detector sum in the Gram form (order S, f = 1)
    bool hs2 = false;                           // order P, split, cropped windows: H multiplies the S_2
                                                // windows (N_2 rows) and Psi is the shared operand
    bool wgram = false;                         // order P, cropped windows: the detector sum as
                                                // Psi^H (M o sum_t conj(H_t) H_t^T) Psi, M = S_2w^H S_2w
    bool wg_fused = false;                      // split window-Gram form: G formed in the Gram GEMM's
                                                // epilogue (every site at most 32 transitions)
    bool raster = false;                        // window-Gram form with Psi and Y = G Psi taken by M x M
                                                // DFTs over the beam lattice (probes on an aligned raster)
    int rM = 0;                                 // DFT side M of the raster form
    int r_chunk = 0, r_chunks = 0;              // window pixels per DFT block, blocks per site
    std::vector<int> r_res;                     // per probe: (i mod M) + M (j mod M), offsets from probe 0
    int64_t r_perm_off = -1;                    // int offset: beam of each compact slot column q
    int64_t r_pos_off = -1;                     // int offset: compact column of grid slot (b mod M) M + (a mod M)
    bool s1_inverse = false;                    // S_1 retreated with the inverse multislice
    bool s2_retreat = false;                    // S_2 retreated towards the exit (inverse multislice)
    int w1_sc = 0;                              // S_1 windows captured SC with c_k(R_0) folded in (raster
                                                // form, split precision, S-matrices not resident), else 0
    int n_img = 0;                              // elastic companion images
    std::vector<double> img_in, img_out;        // their ring angles (rad; out < 0: band limit)
    int img_desc = -1;                          // descriptor of the images' Gram GEMM
    int64_t img_mask_off = -1;                  // int offset: per band slot, bit d = inside ring d
    int64_t det_mask_off = -1;                  // int offset: per band slot, 1 = EELS detector beam
    int64_t col_ptr_off = -1, col_beam_off = -1;// aperture beams grouped by live column (CSR)
    int n_trans_all = 0;                        // transitions of all sites
    int64_t conv_org_off = -1;                  // per site transition plane: (H row, x0, y0, 0) of its window
    int N2p;                                    // N_2 rounded up to 16 (row length of Z)
    std::vector<int> site_w1, site_w2;          // window index of each site (S_1 group-local, S_2 slice-local)
    std::vector<int> site_ix0, site_iy0;
    std::vector<std::vector<int>> site_probes;  // eligible probes (empty vector + flag = all)
    std::vector<SliceInfo> slices;
    std::vector<Group> groups;                  // processing order: descending slices
    std::vector<Batch> batches;
    std::vector<GemmDesc> descs;
    std::vector<Job> jobs;
    int max_w1, max_w2;
    int n_ckpt = 0;                             // S_1 checkpoints (slots of off_ckpt)
    int64_t mid_elems, mid2_elems, part_elems, scratch_elems;   // per batch maxima
    double gemm_flops = 0, sweep_bytes = 0, sweep_beam_slices = 0;
    float c_scale = 1.0f;                       // probe coefficient pre-scale (FP16 range)

    // device table blob (uploaded at the start of every execute)
    std::vector<int32_t> blob;
    int64_t b1_off, b2_off;       // int4 per beam: (live column, iy, a, b)
    int64_t ident_off;            // 0..P-1
    int64_t band_h_off, band_off_off;
    int64_t dz_off, probes_off;   // doubles (int offsets, 16-byte aligned)
    int64_t dbg_ptr, dbg_rec;     // full-plane capture CSR (diagnostics)
    int64_t descs_off;            // GemmDesc array (int offset, 16-byte aligned)

    // workspace layout (byte offsets)
    size_t off_blob, off_twx, off_twy, off_T, off_P, off_C, off_s1, off_s2, off_w1, off_w2,
        off_mid, off_mid2, off_scratch, off_part, off_gtot, off_qpart, off_img_exit, off_img_masked, off_img_part,
        off_img_G, off_img_qpart, off_img_C, off_r_c0, off_r_tw, off_ckpt, ws_bytes;
};

eels_status build_plan(Plan& p, const eels_problem& prob);
uint64_t s_signature(const Plan& p);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;
constexpr int KPAD_MULT = 16;

}  // namespace eels
