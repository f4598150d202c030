// C ABI: plan lifecycle, the device orchestration of one EELS map, and diagnostics.
//
// Order of work for one map (all on the caller's stream):
//   set-up      twiddles, T_j = exp(i sigma V_j), P_j, probe coefficients c_k(R)
//   per group   forward sweep of S_1 from slice 0 to the group's highest ionised slice,
//               capturing the S_1 windows of the group's ionised slices; then the
//               transposed sweep of S_2 continues downward through the group, and at each
//               ionised slice the captured windows are contracted (two grouped GEMMs and a
//               deterministic FP64 reduction into the map).
// Because the S_1 windows of a group are kept, S_2 needs one pass over the slices in
// total instead of being rebuilt for every slice (Sec. 3 rebuilds it per slice).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "eels.h"
#include "internal.h"
#include "kernels.h"

struct eels_plan {
    eels::Plan p;
};

namespace eels {

static thread_local std::string g_err;
void set_error(const std::string& m) { g_err = m; }

static std::atomic<int> g_tune[TUNE_COUNT] = {{2}, {2}, {0}, {1}, {1}, {1}, {1}, {1}, {1}, {1}, {0}, {1}};
int tune_get(int key) { return (key >= 0 && key < TUNE_COUNT) ? g_tune[key].load() : 0; }

// Diagnostic phase timing (eels_timing_enable / eels_timing_read).
struct Timing {
    std::vector<hipEvent_t> ev;   // 2 per group
    std::vector<int> phase;
    int used = 0;
    int cap = 0;
} g_timing;

struct TimeScope {
    int idx = -1;
    hipStream_t st;
    TimeScope(int ph, hipStream_t s) : st(s) {
        if (g_timing.cap > 0 && g_timing.used < g_timing.cap) {
            idx = g_timing.used++;
            g_timing.phase[idx] = ph;
            hipEventRecord(g_timing.ev[2 * idx], st);
        }
    }
    ~TimeScope() {
        if (idx >= 0) hipEventRecord(g_timing.ev[2 * idx + 1], st);
    }
};

#define HIPCHK(x)                                                                       \
    do {                                                                                \
        hipError_t e_ = (x);                                                            \
        if (e_ != hipSuccess) {                                                         \
            set_error(std::string(#x) + ": " + hipGetErrorString(e_));                  \
            return EELS_ERR_DEVICE;                                                     \
        }                                                                               \
    } while (0)

namespace {

struct Dev {
    char* ws;
    const int* blob;
    const int4* b1;
    const int4* b2;
    const double* dz;
    const double* probes;
    const GemmDesc* descs;
    const int *band_h, *band_off;
    float2 *twx, *twy, *T, *P, *C, *s1, *s2, *w1, *w2, *mid, *mid2, *scratch;
    float* part;
    double* gtot;     // Gram form: sum of Z^H Z, FP64 complex [N_1][N_1]
    double* qpart;    // Gram form: per-probe partial quadratic forms
    float2 *img_exit, *img_masked, *img_part, *img_C;   // companion images
    double *img_G, *img_qpart;
    float2 *r_c0, *r_tw;                                  // raster form: c_k(R_0), M-point twiddles
    float2* ckpt;                                         // S_1 checkpoint slots
};

Dev make_dev(const Plan& p, void* ws_) {
    Dev d{};
    d.ws = (char*)ws_;
    d.blob = (const int*)(d.ws + p.off_blob);
    d.b1 = (const int4*)(d.blob + p.b1_off);
    d.b2 = (const int4*)(d.blob + p.b2_off);
    d.dz = (const double*)(d.blob + p.dz_off);
    d.probes = (const double*)(d.blob + p.probes_off);
    d.descs = (const GemmDesc*)(d.blob + p.descs_off);
    d.band_h = d.blob + p.band_h_off;
    d.band_off = d.blob + p.band_off_off;
    d.twx = (float2*)(d.ws + p.off_twx);
    d.twy = (float2*)(d.ws + p.off_twy);
    d.T = (float2*)(d.ws + p.off_T);
    d.P = (float2*)(d.ws + p.off_P);
    d.C = (float2*)(d.ws + p.off_C);
    d.s1 = (float2*)(d.ws + p.off_s1);
    d.s2 = (float2*)(d.ws + p.off_s2);
    d.w1 = (float2*)(d.ws + p.off_w1);
    d.w2 = (float2*)(d.ws + p.off_w2);
    d.mid = (float2*)(d.ws + p.off_mid);
    d.mid2 = (float2*)(d.ws + p.off_mid2);
    d.scratch = (float2*)(d.ws + p.off_scratch);
    d.part = (float*)(d.ws + p.off_part);
    d.gtot = (double*)(d.ws + p.off_gtot);
    d.qpart = (double*)(d.ws + p.off_qpart);
    d.img_exit = (float2*)(d.ws + p.off_img_exit);
    d.img_masked = (float2*)(d.ws + p.off_img_masked);
    d.img_part = (float2*)(d.ws + p.off_img_part);
    d.img_C = (float2*)(d.ws + p.off_img_C);
    d.img_G = (double*)(d.ws + p.off_img_G);
    d.img_qpart = (double*)(d.ws + p.off_img_qpart);
    d.r_c0 = (float2*)(d.ws + p.off_r_c0);
    d.r_tw = (float2*)(d.ws + p.off_r_tw);
    d.ckpt = (float2*)(d.ws + p.off_ckpt);
    return d;
}

eels_status check_ws(const Plan& p, void* ws, size_t bytes) {
    if (!ws || bytes < p.ws_bytes) {
        set_error("workspace smaller than eels_plan_workspace_bytes");
        return EELS_ERR_WORKSPACE;
    }
    if (((uintptr_t)ws) & 255) {
        set_error("workspace must be 256-byte aligned");
        return EELS_ERR_WORKSPACE;
    }
    return EELS_OK;
}

eels_status setup(const Plan& p, const Dev& d, const float* dV, hipStream_t st, bool upload = true) {
    TimeScope ts(EELS_PHASE_SETUP, st);
    if (upload)
        HIPCHK(hipMemcpyAsync((void*)d.blob, p.blob.data(), p.blob.size() * 4, hipMemcpyHostToDevice, st));
    launch_twiddles(d.twx, p.nx, st);
    launch_twiddles(d.twy, p.ny, st);
    launch_transmission(d.T, dV, (int64_t)p.nz * p.ny * p.nx, p.sigma, st);
    launch_propagator(d.P, d.dz, p, st);
    if (p.raster) {
        launch_twiddles(d.r_tw, p.rM, st);
        launch_probe_coefficients(d.r_c0, d.b1, d.probes, p, 0, st, 1);   // c_k(R_0), R_0 = the first probe
    }
    return EELS_OK;
}

const float2* Tj(const Plan& p, const Dev& d, int j) { return d.T + (int64_t)j * p.ny * p.nx; }
// slice j's propagator factor tables (nlx column factors, then ny row factors)
const float2* Pj(const Plan& p, const Dev& d, int j) { return d.P + (int64_t)j * (p.nlx + p.ny); }

// The S_1 windows' storage: complex64, or (raster form in split precision) SC with each beam's
// c_k(R_0) folded in, which makes them the Z product's operand as captured.
void s1_capture_format(const Plan& p, const Dev& d, RowPassArgs& a) {
    a.sc = p.w1_sc;
    a.cfac = p.w1_sc ? d.r_c0 : nullptr;
}

// Forward sweep of S_1 through slices 0..j_end (row pass of j_end included, its column
// pass not).  Captures the windows of the ionised slices of `group` (if >= 0), or the
// full real-space S_1(dbg_slice) into dbg_out.  With exit_cap (j_end = n_z - 1) the last
// column pass also runs and captures the band coefficients of the exit wave
// P_{nz-1} fft2(T_{nz-1} psi) of every beam into exit_cap [N_1][Kb pad].
// A group with a checkpoint slot resumes from S_1 at the entrance of its lowest slice, which
// the first group's sweep saved there (slices[j].ckpt_save) on its way up.
void forward_sweep(const Plan& p, const Dev& d, int j_end, int group, int dbg_slice, float2* dbg_out,
                   hipStream_t st, float2* exit_cap = nullptr, bool last_col = false) {
    TimeScope ts(EELS_PHASE_SWEEP, st);
    const int64_t state = (int64_t)p.N1 * p.ny * p.ldx;
    const int64_t slot = (int64_t)ceil_div(8 * state, 256) * 256 / 8;   // a slot's complex elements
    const int ck = group >= 0 && !dbg_out ? p.groups[group].ckpt : -1;
    const int j_begin = ck >= 0 ? p.groups[group].j_lo : 0;
    if (ck >= 0) launch_copy(d.s1, d.ckpt + ck * slot, state, st);
    else launch_init_forward(d.s1, d.b1, p, st);
    for (int j = j_begin; j <= j_end; ++j) {
        if (group == 0 && !dbg_out && p.slices[j].ckpt_save >= 0)
            launch_copy(d.ckpt + p.slices[j].ckpt_save * slot, d.s1, state, st);
        RowPassArgs a{d.s1, p.N1, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, d.w1, p.N1, p.Kpad, 0,
                      p.ldx};
        if (dbg_out && j == dbg_slice) {
            a.cap_ptr = d.blob + p.dbg_ptr;
            a.cap_rec = d.blob + p.dbg_rec;
            a.win = dbg_out;
            a.Kpad = p.nx * p.ny;
        } else if (group >= 0 && p.slices[j].ion && p.slices[j].group == group) {
            a.cap_ptr = d.blob + p.slices[j].cap1_ptr;
            a.cap_rec = d.blob + p.slices[j].cap1_rec;
            s1_capture_format(p, d, a);
        }
        launch_row_pass(p.nx, 0, a, st);
        if (j < j_end) launch_col_pass(p.ny, 0, d.s1, p.N1, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
        else if (exit_cap || last_col)
            launch_col_pass(p.ny, 0, d.s1, p.N1, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h,
                            exit_cap ? BandCap{d.band_h, d.band_off, exit_cap, p.Kbpad, 0} : BandCap{}, st);
    }
}

// One step of the inverse multislice (Sec. 4.C): S_1 from the entrance of slice j+1 back to
// the entrance of slice j, x_j = F conj(T_j) F^-1 conj(P_j) x_{j+1}, capturing the windows of
// slice j's sites when `capture`.
void inverse_step(const Plan& p, const Dev& d, int j, bool capture, hipStream_t st) {
    TimeScope ts(EELS_PHASE_SWEEP, st);
    launch_col_pass(p.ny, 2, d.s1, p.N1, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
    RowPassArgs a{d.s1, p.N1, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, d.w1, p.N1, p.Kpad, 0,
                  p.ldx};
    if (capture) {
        a.cap_ptr = d.blob + p.slices[j].cap1_ptr;
        a.cap_rec = d.blob + p.slices[j].cap1_rec;
        s1_capture_format(p, d, a);
    }
    launch_row_pass(p.nx, 2, a, st);
}

// One slice of the S_2 retreat (Sec. 4.C applied to S_2) beside the forward S_1 sweep.  With
// `rows`, both row passes of slice j: S_1's (capturing the windows of slice j's sites when
// `capture`) and the inverse of the transposed step's row pass, FFT_x -> (capture S_2(j), the
// value the transposed sweep captures there) -> * conj(T_j) -> iFFT_x.  At slice 0 the state is
// the transposed sweep's before its last row pass, and that pass's capture is taken instead
// (mode 4: the state comes back times nx^2, the scale the inverse row pass leaves).  Otherwise
// both column passes: S_1 to the entrance of slice j+1 and S_2 back to where the transposed
// sweep stood after slice j+1 (iFFT_y -> * conj(P_j) / (nx ny) -> FFT_y).
void retreat_step(const Plan& p, const Dev& d, int j, bool capture, bool rows, hipStream_t st) {
    TimeScope ts(EELS_PHASE_SWEEP, st);
    if (!rows) {
        launch_col_pass(p.ny, 0, d.s1, p.N1, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
        launch_col_pass(p.ny, 3, d.s2, p.N2, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
        return;
    }
    RowPassArgs a{d.s1, p.N1, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, d.w1, p.N1, p.Kpad, 0,
                  p.ldx};
    RowPassArgs b{d.s2, p.N2, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, d.w2 + p.slice_w2[j], p.N2,
                  p.Kpad, p.w2_sc, p.ldx};
    if (capture) {
        a.cap_ptr = d.blob + p.slices[j].cap1_ptr;
        a.cap_rec = d.blob + p.slices[j].cap1_rec;
        s1_capture_format(p, d, a);
        b.cap_ptr = d.blob + p.slices[j].cap2_ptr;
        b.cap_rec = d.blob + p.slices[j].cap2_rec;
    }
    launch_row_pass(p.nx, 0, a, st);
    launch_row_pass(p.nx, j == 0 ? 4 : 3, b, st);
}

// One step of the transposed sweep: bring S_2 to slice j (from j+1, or start at n_z-1)
// and capture what the contraction at j needs: the S_2 windows (real-space contraction,
// in the row pass) or the band coefficients of P_j x_{j+1} (band basis, in the column
// pass or at the start); dbg_out receives the full real-space S_2(j) instead.
void reverse_step(const Plan& p, const Dev& d, int j, bool capture, float2* dbg_out, hipStream_t st) {
    TimeScope ts(EELS_PHASE_SWEEP, st);
    const bool band = capture && p.recip && !dbg_out;
    float2* w2j = d.w2 + p.slice_w2[j];   // this slice's S_2 capture (resident plans keep one per slice)
    if (j == p.nz - 1) {
        launch_init_reverse(d.s2, d.b2, p, st);
        if (band) launch_init_band(w2j, p.Kbpad, d.b2, d.band_h, d.band_off, p, p.w2_sc, st);
    } else {
        BandCap bc{};
        if (band) bc = BandCap{d.band_h, d.band_off, w2j, p.Kbpad, p.w2_sc};
        launch_col_pass(p.ny, 1, d.s2, p.N2, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, bc, st);
    }
    RowPassArgs a{d.s2, p.N2, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, w2j, p.N2, p.Kpad, p.w2_sc,
                  p.ldx};
    if (dbg_out) {
        a.cap_ptr = d.blob + p.dbg_ptr;
        a.cap_rec = d.blob + p.dbg_rec;
        a.win = dbg_out;
        a.Kpad = p.nx * p.ny;
        a.sc = 0;
    } else if (capture && !p.recip) {
        a.cap_ptr = d.blob + p.slices[j].cap2_ptr;
        a.cap_rec = d.blob + p.slices[j].cap2_rec;
    }
    launch_row_pass(p.nx, 1, a, st);
}

// Producer jobs of a batch: the H-multiplied second operand of every site into mid2.
void run_jobs(const Plan& p, const Dev& d, const float2* dH, const Batch& b, int j, hipStream_t st) {
    TimeScope ts(EELS_PHASE_PRODUCER, st);
    for (int k = 0; k < b.job_count; ++k) {
        const Job& jb = p.jobs[b.job_begin + k];
        const float2* W = (jb.from_mid == 2 ? d.w2 : jb.from_mid ? d.mid : d.w1) + jb.w_off;
        if (p.recip) {
            BandFft a{};
            a.dst = d.mid2 + jb.dst_off;
            a.dstride = p.Kbpad;
            a.Kb = p.Kb;
            a.W = W;
            a.wstride = p.Kpad;
            a.Ni = jb.Ni; a.nt = jb.nt; a.ny = p.ny; a.nlx = p.nlx; a.hlx = p.hlx;
            a.Tj = Tj(p, d, j);
            a.H = dH + jb.h_off;
            a.hstride = p.K;
            a.twx = d.twx; a.twy = d.twy;
            a.band_h = d.band_h; a.band_off = d.band_off;
            a.scratch = d.scratch;
            a.ldx = p.ldx;
            a.sc = p.mid2_sc;
            launch_band_fft(p.nx, p.ny, a, st);
        } else {
            launch_hmul(d.mid2 + jb.dst_off, W, p.Kpad, dH + jb.h_off, p.K, jb.Ni, jb.nt, p.K, p.Kpad, p.mid2_sc, st);
        }
    }
}

// Operands of a batch's split-precision GEMMs as contract launches them: epilogue, A and B
// bases, and the store (C) or partial-sum (P) target.  The descriptors' offsets are relative
// to these bases.
struct SplitCall {
    int epi;
    const void *A, *B;
    void* C;
    float* P;
};
SplitCall split_gemm1(const Plan& p, const Dev& d) {
    if (p.gram) return {0, d.mid2, d.w2, d.mid, nullptr};                  // Z = (H S_1) S_2^T
    if (p.order == EELS_ORDER_S_FIRST) return {0, d.w2, d.mid2, d.mid, nullptr};
    return {p.hs2 ? 0 : 3, d.C, d.mid2, d.mid, nullptr};                    // Psi = C S_1w
}
SplitCall split_gemm2(const Plan& p, const Dev& d) {
    if (p.gram) return {2, d.mid, d.mid, nullptr, d.part};                 // Gram tiles of Z
    if (p.order == EELS_ORDER_S_FIRST) return {1, d.mid, d.C, nullptr, d.part};
    if (p.hs2) return {1, d.mid2, d.mid, nullptr, d.part};                 // (H S_2w) Psi
    return {1, d.w2, d.mid2, nullptr, d.part};
}

// Producers a batch needs before its first GEMM: the H-multiplied operand (order S, Gram
// form), or the SC transposes of the S_1 windows (order P in split precision).
void producers_before_gemm1(const Plan& p, const Dev& d, const float2* dH, const Batch& b, hipStream_t st) {
    const bool split = p.precision != EELS_FP32;
    if (p.gram || p.order == EELS_ORDER_S_FIRST) {
        if (split || p.recip) run_jobs(p, d, dH, b, b.slice, st);
    } else if (split && !p.raster) {
        // SC transposes of the sites' S_1 windows (mid2 holds them until the producer runs)
        TimeScope ts(EELS_PHASE_PRODUCER, st);
        if (p.wgram) {   // one launch over the batch (the transposes sit where S_2w^T goes later)
            launch_window_t_batched(d.mid2, d.w1, (const ProdJob*)(d.blob + b.p_jobs), b.job_count, 2, p.Kpad, p.N1,
                                    p.K, p.N1pad, p.precision, nullptr, st);
            return;
        }
        for (int k = 0; k < b.job_count; ++k) {
            const Job& jb = p.jobs[b.job_begin + k];
            launch_window_t_sc(d.mid2 + jb.dst_off, d.w1 + jb.win_off, p.Kpad, p.N1, p.K, p.N1pad, p.precision, st);
        }
    }
}

// ... and between the two GEMMs (order P: the H-multiplied operand from Psi or S_2w).
void producers_after_gemm1(const Plan& p, const Dev& d, const float2* dH, const Batch& b, hipStream_t st) {
    const bool split = p.precision != EELS_FP32;
    if (p.wgram) {
        // window-Gram form, one launch per producer over the batch's sites: each site's S_2 window
        // [N_2][K] becomes rows [K][N_2p] (SC, or complex64 in FP32); in the raster form the S_1
        // window is also transposed into beam-slot order (complex64, the DFTs' input) and, in split
        // precision, copied to SC (the Z GEMM's B operand)
        TimeScope ts(EELS_PHASE_PRODUCER, st);
        const ProdJob* jobs = (const ProdJob*)(d.blob + b.p_jobs);
        launch_window_t_batched(d.mid2, d.w2, jobs, b.job_count, 0, p.Kpad, p.N2, p.K, p.N2p, p.precision, nullptr, st);
        if (p.raster) {
            // split precision: c_k(R_0) folded into Xt and into the Z GEMM's operand
            const bool copy = split && !p.w1_sc;   // SC windows are the Z operand already
            launch_window_t_batched(d.mid2, d.w1, jobs, b.job_count, 1, p.Kpad, p.N1, p.K, p.N1pad, EELS_FP32,
                                    d.blob + p.r_perm_off, st, copy ? p.precision : 0, p.Kpad,
                                    copy ? d.r_c0 : nullptr, p.w1_sc);
        }
        return;
    }
    if (!p.gram && p.order != EELS_ORDER_S_FIRST && (split || p.recip)) run_jobs(p, d, dH, b, b.slice, st);
}

// Window-Gram form of the second product: M = S_2w^H S_2w per site (Gram tiles), G = M o
// sum_t conj(H_t) H_t^T, Y^T = Psi G^T, and the per-probe dot products Re(Psi^H Y).  Split
// precisions keep S_2w^T, G and Psi in SC storage; FP32 keeps them in complex64 and runs the
// FP32 GEMM for the Gram tiles and for G Psi.
void wgram_contract(const Plan& p, const Dev& d, const float2* dH, const Batch& b, hipStream_t st) {
    const int nst = tune_get(TUNE_SC_STAGES);
    // G's diagonal is about N_2 sum_t |H_t|^2 (unit-modulus S_2 rows): scale it by an exact power
    // of two into the FP16 range, and the dot products back
    const float gscale = std::ldexp(1.0f, -(int)std::ceil(std::log2((double)std::max(p.N2, 1))));
    const bool split = p.precision != EELS_FP32;
    {
        TimeScope ts(EELS_PHASE_GRAM, st);
        if (p.wg_fused)   // G straight from the Gram tiles' epilogue
            launch_cgemm_sc(p.precision, 4, nst, d.descs + b.dm_begin, b.dm_count, b.dm_tiles, d.mid2, d.mid2, d.mid2,
                            nullptr, d.blob, st, b.dm_rows, nullptr, dH, gscale);
        else if (split)
            launch_cgemm_sc(p.precision, 2, nst, d.descs + b.dm_begin, b.dm_count, b.dm_tiles, d.mid2, d.mid2, nullptr,
                            (float*)d.mid2, d.blob, st, GEMM_BM);
        else
            launch_cgemm(EELS_FP32, 0, 2, d.descs + b.dm_begin, b.dm_count, b.dm_tiles, d.mid2, d.mid2, nullptr, nullptr,
                         (float*)d.mid2, d.blob, st);
    }
    if (!p.wg_fused) {
        TimeScope ts(EELS_PHASE_PRODUCER, st);
        launch_wgram_combine_batched(d.mid2, dH, (const ProdJob*)(d.blob + b.p_jobs), b.job_count, p.K, p.Kpad, p.Kpad,
                                     gscale, p.precision, st);
    }
    if (p.raster) {
        {
            // Z = G S_1w^T, the window's beams gathered into slot order (from the SC windows as
            // captured, or from their SC copy in mid2)
            TimeScope ts(EELS_PHASE_GEMM2, st);
            if (split)
                launch_cgemm_sc(p.precision, 3, nst, d.descs + b.dy_begin, b.dy_count, b.dy_tiles, d.mid2,
                                p.w1_sc ? (const void*)d.w1 : (const void*)d.mid2, d.mid2, nullptr, d.blob, st,
                                b.dy_rows);
            else
                launch_cgemm(EELS_FP32, 0, 0, d.descs + b.dy_begin, b.dy_count, b.dy_tiles, d.mid2, d.w1, nullptr,
                             d.mid2, nullptr, d.blob, st);
        }
        TimeScope ts(EELS_PHASE_RASTER, st);
        launch_raster_dot((const RasterJob*)(d.blob + b.r_jobs), b.job_count, d.mid2, d.r_c0, d.blob + p.r_perm_off,
                          d.blob + p.r_pos_off, p.rM, p.K, p.N1pad, p.r_chunk, 1.0f / gscale, d.r_tw, d.part, st,
                          split);
        return;
    }
    {
        TimeScope ts(EELS_PHASE_GEMM2, st);
        if (split)
            launch_cgemm_sc(p.precision, 3, nst, d.descs + b.dy_begin, b.dy_count, b.dy_tiles, d.mid, d.mid2, d.mid2,
                            nullptr, d.blob, st, b.dy_rows);
        else
            launch_cgemm(EELS_FP32, 0, 0, d.descs + b.dy_begin, b.dy_count, b.dy_tiles, d.mid, d.mid2, nullptr, d.mid2,
                         nullptr, d.blob, st);
    }
    {
        TimeScope ts(EELS_PHASE_REDUCE, st);
        for (int k = 0; k < b.job_count; ++k) {
            const Job& jb = p.jobs[b.job_begin + k];
            launch_wgram_dot(d.part + jb.part_off, d.mid + jb.psi_off, d.mid2 + jb.y_off, jb.ps, p.K, p.Kpad,
                             1.0f / gscale, p.precision, st);
        }
    }
}

// The batch's partial sums into the map (direct detector sum) or into G (Gram form).
void reduce_batch(const Plan& p, const Dev& d, double* map, const Batch& b, hipStream_t st) {
    TimeScope ts(EELS_PHASE_REDUCE, st);
    if (p.gram) {
        launch_gram_reduce(d.gtot, (const float2*)d.part, b.n_parts, (int64_t)p.N1pad * p.N1pad, p.N1, p.N1pad, st);
        return;
    }
    double nn = (double)p.nx * (double)p.ny;
    double scale = (double)p.f * p.f / (nn * nn) / ((double)p.c_scale * p.c_scale);
    if (b.red_ptr < 0) launch_reduce_dense(map, p.P, d.descs, b.d2_begin, b.d2_count, d.part, scale, st);
    else launch_reduce(map, p.P, d.blob + b.red_ptr, d.blob + b.red_ent, d.descs, d.part, scale, st);
}

void contract(const Plan& p, const Dev& d, const float2* dH, double* map, int bi, hipStream_t st) {
    const Batch& b = p.batches[bi];
    const GemmDesc* dd = d.descs;
    const bool split = p.precision != EELS_FP32;
    const int nst = tune_get(TUNE_SC_STAGES);
    const bool h_pro = !p.recip;   // FP32 real-space: H applied in the GEMM prologue
    const bool orderS = p.order == EELS_ORDER_S_FIRST;
    producers_before_gemm1(p, d, dH, b, st);
    {
        TimeScope ts(EELS_PHASE_GEMM1, st);
        if (split) {
            const SplitCall c = split_gemm1(p, d);
            launch_cgemm_sc(p.precision, c.epi, nst, dd + b.d1_begin, b.d1_count, b.d1_tiles, c.A, c.B, c.C, c.P,
                            d.blob, st, b.d1_rows);
        } else if (p.gram) {
            launch_cgemm(EELS_FP32, 0, 0, dd + b.d1_begin, b.d1_count, b.d1_tiles, d.mid2, d.w2, nullptr, d.mid,
                         nullptr, d.blob, st);
        } else if (orderS) {
            launch_cgemm(EELS_FP32, 0, 0, dd + b.d1_begin, b.d1_count, b.d1_tiles, d.w2, h_pro ? d.w1 : d.mid2,
                         h_pro ? dH : nullptr, d.mid, nullptr, d.blob, st);
        } else {
            launch_cgemm(EELS_FP32, 1, 0, dd + b.d1_begin, b.d1_count, b.d1_tiles, d.C, d.w1, nullptr, d.mid, nullptr,
                         d.blob, st);
        }
    }
    producers_after_gemm1(p, d, dH, b, st);
    if (p.wgram) {
        wgram_contract(p, d, dH, b, st);
        reduce_batch(p, d, map, b, st);
        return;
    }
    {
        TimeScope ts(EELS_PHASE_GEMM2, st);
        if (split) {
            const SplitCall c = split_gemm2(p, d);
            launch_cgemm_sc(p.precision, c.epi, nst, dd + b.d2_begin, b.d2_count, b.d2_tiles, c.A, c.B, c.C, c.P,
                            d.blob, st, b.d2_rows);
        } else if (p.gram) {
            launch_cgemm(EELS_FP32, 0, 2, dd + b.d2_begin, b.d2_count, b.d2_tiles, d.mid, d.mid, nullptr, nullptr,
                         d.part, d.blob, st);
        } else if (orderS) {
            launch_cgemm(EELS_FP32, 0, 1, dd + b.d2_begin, b.d2_count, b.d2_tiles, d.mid, d.C, nullptr, nullptr,
                         d.part, d.blob, st);
        } else {
            launch_cgemm(EELS_FP32, 0, 1, dd + b.d2_begin, b.d2_count, b.d2_tiles, d.w2, h_pro ? d.mid : d.mid2,
                         h_pro ? dH : nullptr, nullptr, d.part, d.blob, st);
        }
    }
    reduce_batch(p, d, map, b, st);
}

// Companion images from the exit-wave band coefficients in img_exit: for each ring d,
// X = the coefficients masked to the ring, G_d = X^H X (FP32 Gram tiles, FP64 sum) and
// I_d(R) = c(R)^H G_d c(R) / c_scale^2 (interp_f = 1).
void companion_images(const Plan& p, const Dev& d, double* images, hipStream_t st) {
    TimeScope ts(EELS_PHASE_IMAGES, st);
    launch_probe_coefficients(d.img_C, d.b1, d.probes, p, 0, st);
    const GemmDesc* dd = d.descs + p.img_desc;
    const int tiles = (int)(ceil_div(p.N1, GEMM_BM) * ceil_div(p.N1, GEMM_BN));
    const double scale = 1.0 / ((double)p.c_scale * p.c_scale);
    for (int k = 0; k < p.n_img; ++k) {
        launch_mask_band(d.img_masked, d.img_exit, p.N1, p.Kbpad, d.blob + p.img_mask_off, 1 << k, st);
        launch_cgemm(EELS_FP32, 0, 2, dd, 1, tiles, d.img_masked, d.img_masked, nullptr, nullptr, (float*)d.img_part,
                     d.blob, st);
        launch_fill_zero_d(d.img_G, 2 * (int64_t)p.N1 * p.N1, st);
        launch_gram_reduce(d.img_G, d.img_part, 1, 0, p.N1, p.N1pad, st);
        launch_fill_zero_d(images + (int64_t)k * p.P, p.P, st);
        launch_quadform(images + (int64_t)k * p.P, p.P, d.img_G, p.N1, d.img_C, p.N1pad, d.img_qpart, scale, st);
    }
}

// Gram form: I(R) = scale * c(R)^H G c(R) once every batch has added its Z^H Z to G.
void finish_map(const Plan& p, const Dev& d, double* map, hipStream_t st) {
    if (!p.gram) return;
    TimeScope ts(EELS_PHASE_REDUCE, st);
    double nn = (double)p.nx * (double)p.ny;
    double scale = (double)p.f * p.f / (nn * nn) / ((double)p.c_scale * p.c_scale);
    launch_quadform(map, p.P, d.gtot, p.N1, d.C, p.N1pad, d.qpart, scale, st);
}

// Workspace of the conventional multislice: its own compact layout (tables, T, P, the
// elastic and inelastic waves of one probe chunk), none of the scattering-matrix buffers.
struct ConvLayout {
    size_t blob, twx, twy, T, P, Hfull, psi, waves, exit_band, wnorm, total;
};

ConvLayout conv_layout(const Plan& p, int chunk) {
    ConvLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += (size_t)round_up((int64_t)std::max<size_t>(bytes, 16), 256); return o; };
    const size_t c8 = 8, plane = (size_t)p.ny * p.ldx;
    const size_t n_inel = (size_t)chunk * p.n_trans_all;
    L.blob = take(p.blob.size() * 4);
    L.twx = take(c8 * p.nx);
    L.twy = take(c8 * p.ny);
    L.T = take(c8 * (size_t)p.nz * p.ny * p.nx);
    L.P = take(c8 * (size_t)p.nz * (p.nlx + p.ny));
    L.Hfull = take(p.full_window ? 16 : c8 * (size_t)p.n_trans_all * p.ny * p.nx);
    L.psi = take(c8 * (size_t)chunk * p.ny * p.nx);
    L.waves = take(c8 * ((size_t)chunk + n_inel) * plane);
    L.exit_band = take(c8 * n_inel * p.Kbpad);
    L.wnorm = take(8 * n_inel);
    L.total = off;
    return L;
}

}  // namespace
}  // namespace eels

using namespace eels;

extern "C" {

eels_status eels_get_version(int* major, int* minor) {
    if (major) *major = EELS_VERSION_MAJOR;
    if (minor) *minor = EELS_VERSION_MINOR;
    return EELS_OK;
}

const char* eels_status_string(eels_status s) {
    switch (s) {
        case EELS_OK: return "ok";
        case EELS_ERR_INVALID_ARG: return "invalid argument";
        case EELS_ERR_BANDLIMIT: return "beam outside the band limit";
        case EELS_ERR_UNSUPPORTED_SIZE: return "unsupported grid size";
        case EELS_ERR_WORKSPACE: return "workspace too small";
        case EELS_ERR_OOM: return "does not fit the memory budget";
        case EELS_ERR_DEVICE: return "device error";
        case EELS_ERR_CANCELLED: return "cancelled";
        default: return "internal error";
    }
}

const char* eels_last_error(void) { return g_err.c_str(); }

eels_status eels_plan_create(eels_plan** out, const eels_problem* prob) {
    if (!out || !prob) {
        set_error("null argument");
        return EELS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    try {
        eels_plan* pl = new eels_plan;
        eels_status s = build_plan(pl->p, *prob);
        if (s != EELS_OK) {
            delete pl;
            return s;
        }
        *out = pl;
        return EELS_OK;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed while planning");
        return EELS_ERR_OOM;
    } catch (...) {
        set_error("unexpected exception while planning");
        return EELS_ERR_INTERNAL;
    }
}

eels_status eels_plan_workspace_bytes(const eels_plan* p, size_t* bytes) {
    if (!p || !bytes) return EELS_ERR_INVALID_ARG;
    *bytes = p->p.ws_bytes;
    return EELS_OK;
}

eels_status eels_plan_info_get(const eels_plan* pl, eels_plan_info* info) {
    if (!pl || !info) return EELS_ERR_INVALID_ARG;
    const Plan& p = pl->p;
    std::memset(info, 0, sizeof(*info));
    info->n_beams_in = p.N1;
    info->n_beams_out = p.N2;
    info->n_beams_in_fine = p.N1fine;
    info->n_live_x = p.nlx;
    info->window_nx = p.nwx;
    info->window_ny = p.nwy;
    info->k_pixels = p.K;
    info->k_stride = p.Kpad;
    int nion = 0;
    for (auto& s : p.slices) nion += s.ion ? 1 : 0;
    info->n_ion_slices = nion;
    info->n_groups = (int)p.groups.size();
    info->n_batches = (int)p.batches.size();
    info->order = p.order;
    info->band_basis = p.recip ? 1 : 0;
    info->band_pixels = p.Kb;
    info->window_gram_form = p.wgram ? 1 : 0;
    info->raster_form = p.raster ? p.rM : 0;
    info->n_checkpoints = p.n_ckpt;
    info->lambda_A = p.lam;
    info->sigma = p.sigma;
    info->gemm_flops = p.gemm_flops;
    info->sweep_bytes = p.sweep_bytes;
    info->sweep_beam_slices = p.sweep_beam_slices;
    info->workspace_bytes = p.ws_bytes;
    info->gram_form = p.gram ? 1 : 0;
    return EELS_OK;
}

eels_status eels_plan_beams(const eels_plan* pl, int which, int* ab, int count) {
    if (!pl || !ab || (which != 0 && which != 1)) return EELS_ERR_INVALID_ARG;
    const auto& v = which == 0 ? pl->p.ab1 : pl->p.ab2;
    if (count < (int)v.size() / 2) return EELS_ERR_INVALID_ARG;
    std::memcpy(ab, v.data(), v.size() * sizeof(int));
    return EELS_OK;
}

eels_status eels_plan_destroy(eels_plan* p) {
    delete p;
    return EELS_OK;
}

eels_status eels_execute(const eels_plan* pl, const float* d_V, const void* d_H, double* d_map, void* d_workspace,
                         size_t workspace_bytes, void* stream) {
    return eels_execute_ex(pl, d_V, d_H, d_map, d_workspace, workspace_bytes, stream, 0u);
}

eels_status eels_execute_ex(const eels_plan* pl, const float* d_V, const void* d_H, double* d_map, void* d_workspace,
                            size_t workspace_bytes, void* stream, unsigned flags) {
    return eels_execute_images(pl, d_V, d_H, d_map, nullptr, d_workspace, workspace_bytes, stream, flags);
}

eels_status eels_execute_images(const eels_plan* pl, const float* d_V, const void* d_H, double* d_map,
                                double* d_images, void* d_workspace, size_t workspace_bytes, void* stream,
                                unsigned flags) {
    if (!pl || !d_V || !d_map) {
        set_error("null argument");
        return EELS_ERR_INVALID_ARG;
    }
    const Plan& p = pl->p;
    if (p.n_trans_total > 0 && !d_H) {
        set_error("transition potentials missing");
        return EELS_ERR_INVALID_ARG;
    }
    if (flags & ~(unsigned)(EELS_EXEC_SKIP_UPLOAD | EELS_EXEC_SKIP_SWEEPS | EELS_EXEC_SWEEPS_ONLY)) {
        set_error("unknown execute flag");
        return EELS_ERR_INVALID_ARG;
    }
    const bool skip_sweeps = (flags & EELS_EXEC_SKIP_SWEEPS) != 0;
    const bool sweeps_only = (flags & EELS_EXEC_SWEEPS_ONLY) != 0;
    if ((skip_sweeps || sweeps_only) && !p.resident) {
        set_error("EELS_EXEC_SKIP_SWEEPS and EELS_EXEC_SWEEPS_ONLY need a plan with resident_s");
        return EELS_ERR_INVALID_ARG;
    }
    if (skip_sweeps && sweeps_only) {
        set_error("EELS_EXEC_SKIP_SWEEPS and EELS_EXEC_SWEEPS_ONLY exclude each other");
        return EELS_ERR_INVALID_ARG;
    }
    if (sweeps_only && d_images && p.n_img > 0) {
        set_error("EELS_EXEC_SWEEPS_ONLY does not compute companion images");
        return EELS_ERR_INVALID_ARG;
    }
    eels_status s = check_ws(p, d_workspace, workspace_bytes);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    Dev d = make_dev(p, d_workspace);
    g_timing.used = 0;
    if ((s = setup(p, d, d_V, st, !(flags & EELS_EXEC_SKIP_UPLOAD)))) return s;
    launch_probe_coefficients(d.C, d.b1, d.probes, p, p.c_sc, st);
    launch_fill_zero_d(d_map, p.P, st);
    if (p.gram) launch_fill_zero_d(d.gtot, 2 * (int64_t)p.N1 * p.N1, st);
    const bool images = d_images && p.n_img > 0;
    if (images && (skip_sweeps || p.groups.empty())) {
        // no forward sweep runs below (resident S-matrices, or no sites): sweep for the images
        forward_sweep(p, d, p.nz - 1, -1, -1, nullptr, st, d.img_exit);
        companion_images(p, d, d_images, st);
    }
    if (skip_sweeps) {
        // the S_1 windows and every slice's S_2 capture are already in the workspace
        for (int j = p.nz - 1; j >= 0; --j)
            if (p.slices[j].ion)
                for (int bi : p.slices[j].batches) contract(p, d, (const float2*)d_H, d_map, bi, st);
        finish_map(p, d, d_map, st);
        HIPCHK(hipGetLastError());
        return EELS_OK;
    }
    // split operands are read in whole 16-element K tiles: the S_2 capture's padding must be zero,
    // and so must the SC S_1 windows' (the captures write pixels 0 .. K-1 of every row)
    if (p.precision != EELS_FP32) launch_fill_zero(d.w2, p.off_C - p.off_w2, st);
    if (p.w1_sc) launch_sc_zero_cols(d.w1, (int64_t)std::max(p.max_w1, 1) * p.N1, p.Kpad, p.K, st);
    if (p.s1_inverse && !p.groups.empty()) {
        // S_1 through every slice to the exit (capturing the exit wave for the images), then
        // back down with the inverse multislice beside the transposed S_2 sweep
        forward_sweep(p, d, p.nz - 1, -1, -1, nullptr, st, images ? d.img_exit : nullptr, true);
        if (images) companion_images(p, d, d_images, st);
        for (int j = p.nz - 1; j >= p.groups[0].j_lo; --j) {
            reverse_step(p, d, j, p.slices[j].ion, nullptr, st);
            inverse_step(p, d, j, p.slices[j].ion, st);
            if (p.slices[j].ion)
                for (int bi : p.slices[j].batches) contract(p, d, (const float2*)d_H, d_map, bi, st);
        }
        finish_map(p, d, d_map, st);
        HIPCHK(hipGetLastError());
        return EELS_OK;
    }
    if (p.s2_retreat && !p.groups.empty()) {
        // S_2 through every slice to the entrance, then back up with the inverse of each
        // transposed step beside the forward S_1 sweep, slice by slice up to the top site
        if (images) {
            forward_sweep(p, d, p.nz - 1, -1, -1, nullptr, st, d.img_exit);
            companion_images(p, d, d_images, st);
        }
        for (int j = p.nz - 1; j >= 1; --j) reverse_step(p, d, j, false, nullptr, st);
        const int j_top = p.groups[0].j_hi;
        {
            // the state before the row pass of slice 0 (band-limited, so held exactly)
            TimeScope ts(EELS_PHASE_SWEEP, st);
            if (p.nz == 1) launch_init_reverse(d.s2, d.b2, p, st);
            else launch_col_pass(p.ny, 1, d.s2, p.N2, p.nlx, p.ldx, Pj(p, d, 0), d.twy, d.band_h, BandCap{}, st);
            launch_init_forward(d.s1, d.b1, p, st);
        }
        for (int j = 0; j <= j_top; ++j) {
            retreat_step(p, d, j, p.slices[j].ion, true, st);
            if (p.slices[j].ion)
                for (int bi : p.slices[j].batches) contract(p, d, (const float2*)d_H, d_map, bi, st);
            if (j < j_top) retreat_step(p, d, j, false, false, st);
        }
        finish_map(p, d, d_map, st);
        HIPCHK(hipGetLastError());
        return EELS_OK;
    }
    int rev_next = p.nz - 1;
    for (int gi = 0; gi < (int)p.groups.size(); ++gi) {
        const Group& g = p.groups[gi];
        // the first (highest) group's forward sweep continues to the exit for the images
        const bool exit_here = images && gi == 0;
        forward_sweep(p, d, exit_here ? p.nz - 1 : g.j_hi, gi, -1, nullptr, st, exit_here ? d.img_exit : nullptr);
        if (exit_here) companion_images(p, d, d_images, st);
        for (int j = rev_next; j >= g.j_lo; --j) {
            reverse_step(p, d, j, p.slices[j].ion, nullptr, st);
            if (p.slices[j].ion && !sweeps_only)
                for (int bi : p.slices[j].batches) contract(p, d, (const float2*)d_H, d_map, bi, st);
        }
        rev_next = g.j_lo - 1;
    }
    if (!sweeps_only) finish_map(p, d, d_map, st);
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- allocation-free execution
// A fixed device array stands in for the workspace of eels_execute_noalloc.  Each device the
// library runs on holds its own copy at its own address, found once per device with
// hipGetSymbolAddress; host code uses only that address, never the array's name.
namespace eels {
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
}  // namespace eels
static __device__ __align__(256) unsigned char scratch[eels::NOALLOC_SCRATCH_BYTES];
static void* g_scratch_addr[eels::NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

extern "C" {

eels_status eels_execute_noalloc(const eels_plan* pl, const float* d_V, const void* d_H, double* d_map,
                                 void* stream) {
    if (!pl) {
        set_error("null argument");
        return EELS_ERR_INVALID_ARG;
    }
    if (pl->p.ws_bytes > NOALLOC_SCRATCH_BYTES) {
        set_error("the plan needs " + std::to_string(pl->p.ws_bytes) +
                  " workspace bytes; eels_execute_noalloc holds at most " + std::to_string(NOALLOC_SCRATCH_BYTES));
        return EELS_ERR_WORKSPACE;
    }
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) {
        set_error("device index beyond the allocation-free entry point's table");
        return EELS_ERR_INVALID_ARG;
    }
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch_addr[dev]) {
            void* a = nullptr;
            const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !a) {
                set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
                return EELS_ERR_DEVICE;
            }
            g_scratch_addr[dev] = a;
        }
        ptr = g_scratch_addr[dev];
    }
    // every buffer the map reads is written first by the same call (tables, T, P, sweeps,
    // partial sums, the zeroed S_2 padding), so the previous call's contents do not matter
    return eels_execute_ex(pl, d_V, d_H, d_map, ptr, NOALLOC_SCRATCH_BYTES, stream, 0u);
}

size_t eels_conventional_workspace_bytes(const eels_plan* pl, int probe_chunk) {
    if (!pl || probe_chunk < 1) return 0;
    return conv_layout(pl->p, probe_chunk).total;
}

// Conventional multislice EELS map.  Per chunk of probes, slice by slice:
//   row pass of the elastic waves (capturing their real-space entrance wave psi at an
//     ionised slice) and of the inelastic waves alive so far;
//   at an ionised slice, each site's transitions spawn T_j H_n psi through the row stage
//     of the band FFT (the same result as a row pass of H_n psi), appended to the waves;
//   column pass (x P_j) of all waves; the last slice's captures the exit band of the
//     inelastic waves, whose detector sums give the map.
// The elastic wave stops after the last ionised slice.
eels_status eels_conventional_map(const eels_plan* pl, const float* d_V, const void* d_H, double* d_map,
                                  int probe_chunk, void* d_workspace, size_t workspace_bytes, void* stream) {
    if (!pl || !d_V || !d_map || probe_chunk < 1) {
        set_error("null argument or probe_chunk < 1");
        return EELS_ERR_INVALID_ARG;
    }
    const Plan& p = pl->p;
    if (p.f != 1) {
        set_error("conventional multislice needs interp_f = 1");
        return EELS_ERR_INVALID_ARG;
    }
    if ((p.nx & (p.nx - 1)) || (p.ny & (p.ny - 1))) {
        set_error("conventional multislice needs power-of-two grid sides");
        return EELS_ERR_UNSUPPORTED_SIZE;
    }
    if (p.n_trans_total > 0 && !d_H) {
        set_error("transition potentials missing");
        return EELS_ERR_INVALID_ARG;
    }
    const ConvLayout L = conv_layout(p, probe_chunk);
    if (!d_workspace || workspace_bytes < L.total) {
        set_error("workspace smaller than eels_conventional_workspace_bytes");
        return EELS_ERR_WORKSPACE;
    }
    if (((uintptr_t)d_workspace) & 255) {
        set_error("workspace must be 256-byte aligned");
        return EELS_ERR_WORKSPACE;
    }
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_workspace;
    Dev d{};
    d.ws = ws;
    d.blob = (const int*)(ws + L.blob);
    d.b1 = (const int4*)(d.blob + p.b1_off);
    d.dz = (const double*)(d.blob + p.dz_off);
    d.probes = (const double*)(d.blob + p.probes_off);
    d.band_h = d.blob + p.band_h_off;
    d.band_off = d.blob + p.band_off_off;
    d.twx = (float2*)(ws + L.twx);
    d.twy = (float2*)(ws + L.twy);
    d.T = (float2*)(ws + L.T);
    d.P = (float2*)(ws + L.P);
    float2* psi = (float2*)(ws + L.psi);
    float2* waves = (float2*)(ws + L.waves);
    float2* exit_band = (float2*)(ws + L.exit_band);
    double* wnorm = (double*)(ws + L.wnorm);
    g_timing.used = 0;
    eels_status s = setup(p, d, d_V, st);
    if (s) return s;
    const int64_t plane_nx = (int64_t)p.nx * p.ny, plane = (int64_t)p.ny * p.ldx;
    const float2* Hb = (const float2*)d_H;
    std::vector<int64_t> site_plane(p.sites.size(), 0);   // first H plane of each site
    {
        int64_t acc = 0;
        for (size_t k = 0; k < p.sites.size(); ++k) {
            site_plane[k] = p.full_window ? p.sites[k].h_offset : acc;
            acc += p.sites[k].n_trans;
        }
    }
    if (!p.full_window && p.n_trans_all > 0) {
        TimeScope ts(EELS_PHASE_SETUP, st);
        launch_conv_scatter_h((float2*)(ws + L.Hfull), Hb, d.blob + p.conv_org_off, p.n_trans_all, p, st);
        Hb = (const float2*)(ws + L.Hfull);
    }
    std::vector<std::vector<int>> by_slice(p.nz);
    int j_last = -1;
    for (size_t k = 0; k < p.sites.size(); ++k)
        if (p.sites[k].n_trans > 0) {
            by_slice[p.sites[k].slice].push_back((int)k);
            j_last = std::max(j_last, p.sites[k].slice);
        }
    launch_fill_zero_d(d_map, p.P, st);
    for (int p0 = 0; p0 < p.P && j_last >= 0; p0 += probe_chunk) {
        const int Ni = std::min(probe_chunk, p.P - p0);
        float2* inel = waves + (int64_t)Ni * plane;
        int64_t n_inel = 0;
        {
            TimeScope ts(EELS_PHASE_SWEEP, st);
            launch_conv_init(waves, Ni, p0, p, d.blob + p.col_ptr_off, d.blob + p.col_beam_off, d.b1, d.probes, st);
        }
        for (int j = 0; j < p.nz; ++j) {
            const bool ion = !by_slice[j].empty();
            {
                TimeScope ts(EELS_PHASE_SWEEP, st);
                if (j <= j_last) {
                    RowPassArgs a{waves, Ni, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, psi, Ni,
                                  (int)plane_nx, 0, p.ldx};
                    if (ion) {
                        a.cap_ptr = d.blob + p.dbg_ptr;
                        a.cap_rec = d.blob + p.dbg_rec;
                    }
                    launch_row_pass(p.nx, 0, a, st);
                }
                if (n_inel > 0) {
                    RowPassArgs a{inel, (int)n_inel, p.ny, p.nlx, p.hlx, Tj(p, d, j), d.twx, nullptr, nullptr, nullptr,
                                  0, 0, 0, p.ldx};
                    launch_row_pass(p.nx, 0, a, st);
                }
            }
            if (ion) {
                TimeScope ts(EELS_PHASE_PRODUCER, st);
                for (int k : by_slice[j]) {
                    const int nt = p.sites[k].n_trans;
                    launch_band_rows(inel + n_inel * plane, psi, plane_nx, Ni, nt, p, Tj(p, d, j),
                                     Hb + site_plane[k] * plane_nx, plane_nx, d.twx, st);
                    n_inel += (int64_t)nt * Ni;
                }
            }
            TimeScope ts(EELS_PHASE_SWEEP, st);
            if (j == p.nz - 1) {
                if (n_inel > 0)
                    launch_col_pass(p.ny, 0, inel, (int)n_inel, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h,
                                    BandCap{d.band_h, d.band_off, exit_band, p.Kbpad, 0}, st);
            } else if (j < j_last) {
                launch_col_pass(p.ny, 0, waves, (int)(Ni + n_inel), p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
            } else if (n_inel > 0) {
                launch_col_pass(p.ny, 0, inel, (int)n_inel, p.nlx, p.ldx, Pj(p, d, j), d.twy, d.band_h, BandCap{}, st);
            }
        }
        TimeScope ts(EELS_PHASE_REDUCE, st);
        launch_conv_norm(wnorm, exit_band, p.Kbpad, p.Kb, d.blob + p.det_mask_off, n_inel, st);
        launch_conv_map(d_map + p0, wnorm, Ni, n_inel / Ni, st);
    }
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

eels_status eels_plan_s_signature(const eels_plan* pl, uint64_t* sig) {
    if (!pl || !sig) return EELS_ERR_INVALID_ARG;
    *sig = s_signature(pl->p);
    return EELS_OK;
}

eels_status eels_debug_s1(const eels_plan* pl, const float* d_V, int slice, void* d_out, void* d_workspace,
                          size_t workspace_bytes, void* stream) {
    if (!pl || !d_V || !d_out || slice < 0 || slice >= pl->p.nz) return EELS_ERR_INVALID_ARG;
    const Plan& p = pl->p;
    eels_status s = check_ws(p, d_workspace, workspace_bytes);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    Dev d = make_dev(p, d_workspace);
    if ((s = setup(p, d, d_V, st))) return s;
    forward_sweep(p, d, slice, -1, slice, (float2*)d_out, st);
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

eels_status eels_debug_s2(const eels_plan* pl, const float* d_V, int slice, void* d_out, void* d_workspace,
                          size_t workspace_bytes, void* stream) {
    if (!pl || !d_V || !d_out || slice < 0 || slice >= pl->p.nz) return EELS_ERR_INVALID_ARG;
    const Plan& p = pl->p;
    eels_status s = check_ws(p, d_workspace, workspace_bytes);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    Dev d = make_dev(p, d_workspace);
    if ((s = setup(p, d, d_V, st))) return s;
    for (int j = p.nz - 1; j >= slice; --j) reverse_step(p, d, j, false, j == slice ? (float2*)d_out : nullptr, st);
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

size_t eels_gemm_work_bytes(int m, int n, int k) {
    if (m <= 0 || n <= 0 || k <= 0) return 0;
    size_t kp = (size_t)round_up(k, KPAD_MULT);
    size_t part = (size_t)ceil_div(m, GEMM_BM) * (size_t)n * 4;
    size_t np_ = (size_t)round_up(n, KPAD_MULT);
    size_t tmp = std::max((size_t)std::max(m, n) * kp, (size_t)m * np_);
    size_t sc = ((size_t)m * kp + (size_t)n * kp + (size_t)m * np_ + tmp) * 8;
    return 512 + (size_t)round_up((int64_t)part, 256) + sc + 1024;
}

eels_status eels_debug_cgemm(int precision, int m, int n, int k, const void* d_A, int lda, const void* d_B, int ldb,
                             void* d_C, int ldc, double* d_norm2, void* d_work, void* stream) {
    if (m <= 0 || n <= 0 || k <= 0 || !d_A || !d_B || !d_work || (!d_C && !d_norm2)) return EELS_ERR_INVALID_ARG;
    if (lda < k || ldb < k || (lda & 1) || (ldb & 1) || (d_C && ldc < n)) return EELS_ERR_INVALID_ARG;
    if (precision < EELS_FP32 || precision > EELS_FP16_SPLIT) return EELS_ERR_INVALID_ARG;
    if (((uintptr_t)d_work) & 255) return EELS_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    GemmDesc g{};
    g.a_off = 0; g.lda = lda; g.b_off = 0; g.ldb = ldb;
    g.h_off = -1; g.c_off = 0; g.ldc_m = ldc; g.ldc_t = 0; g.p_off = 0; g.ld_part = n; g.a_tstride = 0;
    g.b_tstride = 0;
    g.M = m; g.N_inner = n; g.n_t = 1; g.K = k; g.idx_off = -1;
    g.tiles_m = (int)ceil_div(m, GEMM_BM);
    g.tiles_n = (int)ceil_div(n, GEMM_BN);
    g.tile_start = 0;
    char* w = (char*)d_work;
    GemmDesc* dd = (GemmDesc*)w;
    float* part = (float*)(w + 512);
    size_t part_bytes = (size_t)round_up((int64_t)g.tiles_m * n * 4, 256);
    int tiles = g.tiles_m * g.tiles_n;
    if (precision == EELS_FP32) {
        HIPCHK(hipMemcpyAsync(dd, &g, sizeof(g), hipMemcpyHostToDevice, st));
        if (d_norm2) {
            launch_cgemm(precision, 0, 1, dd, 1, tiles, (const float2*)d_A, (const float2*)d_B, nullptr, nullptr, part,
                         nullptr, st);
        } else {
            launch_cgemm(precision, 0, 0, dd, 1, tiles, (const float2*)d_A, (const float2*)d_B, nullptr, (float2*)d_C,
                         nullptr, nullptr, st);
        }
    } else {
        // convert the operands to split-complex storage with K padded to 16
        int kp = (int)round_up(k, KPAD_MULT), np_ = (int)round_up(n, KPAD_MULT);
        char* a_sc = w + 512 + part_bytes;
        char* b_sc = a_sc + (size_t)m * kp * 8;
        char* c_sc = b_sc + (size_t)n * kp * 8;
        char* tmp = c_sc + (size_t)m * np_ * 8;
        // strided copy: rows of lda -> rows of kp (via complex64 rows; K columns only)
        g.lda = kp; g.ldb = kp; g.ldc_m = np_;
        HIPCHK(hipMemcpyAsync(dd, &g, sizeof(g), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpy2DAsync(tmp, (size_t)kp * 8, d_A, (size_t)lda * 8, (size_t)k * 8, m, hipMemcpyDeviceToDevice, st));
        launch_to_sc(a_sc, (const float2*)tmp, m, k, kp, precision, st);
        HIPCHK(hipMemcpy2DAsync(tmp, (size_t)kp * 8, d_B, (size_t)ldb * 8, (size_t)k * 8, n, hipMemcpyDeviceToDevice, st));
        launch_to_sc(b_sc, (const float2*)tmp, n, k, kp, precision, st);
        int nst = tune_get(TUNE_SC_STAGES);
        if (d_norm2) {
            launch_cgemm_sc(precision, 1, nst, dd, 1, tiles, a_sc, b_sc, nullptr, part, nullptr, st);
        } else {
            launch_cgemm_sc(precision, 0, nst, dd, 1, tiles, a_sc, b_sc, c_sc, nullptr, nullptr, st);
            launch_from_sc((float2*)tmp, c_sc, (int64_t)m * np_, precision, st);
            HIPCHK(hipMemcpy2DAsync(d_C, (size_t)ldc * 8, tmp, (size_t)np_ * 8, (size_t)n * 8, m,
                                    hipMemcpyDeviceToDevice, st));
        }
    }
    if (d_norm2) {
        launch_fill_zero_d(d_norm2, n, st);
        launch_reduce_dense(d_norm2, n, dd, 0, 1, part, 1.0, st);
    }
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

eels_status eels_tune_set(int key, int value) {
    if (key < 0 || key >= TUNE_COUNT) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_SC_STAGES && (value < 2 || value > 5)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_TILE_ORDER && (value < 0 || value > 2)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_SC_SCHED && (value < 0 || value > 3)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_GRAM_STACK && (value < 0 || value > 1)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_GEMM1_ROWS && (value < 0 || value > 1)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_GEMM2_ROWS && (value < 0 || value > 1)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_WINDOW_GRAM && (value < 0 || value > 2)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_RASTER && (value < 0 || value > 2)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_CHECKPOINT && (value < 0 || value > 2)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_WG_FUSED && (value < 0 || value > 1)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_GRAM_ROWS && (value < 0 || value > 1)) return EELS_ERR_INVALID_ARG;
    if (key == TUNE_GEMM_STAGING && (value < 0 || value > 2)) return EELS_ERR_INVALID_ARG;
    g_tune[key].store(value);
    return EELS_OK;
}

int eels_tune_get(int key) { return tune_get(key); }

eels_status eels_timing_enable(int capacity) {
    if (capacity < 0) return EELS_ERR_INVALID_ARG;
    for (auto e : g_timing.ev) hipEventDestroy(e);
    g_timing.ev.clear();
    g_timing.phase.clear();
    g_timing.used = 0;
    g_timing.cap = 0;
    if (capacity == 0) return EELS_OK;
    g_timing.ev.resize(2 * (size_t)capacity);
    g_timing.phase.assign(capacity, 0);
    for (auto& e : g_timing.ev) HIPCHK(hipEventCreate(&e));
    g_timing.cap = capacity;
    return EELS_OK;
}

eels_status eels_timing_read(double* ms, int* counts) {
    if (!ms || !counts) return EELS_ERR_INVALID_ARG;
    for (int k = 0; k < EELS_PHASES; ++k) { ms[k] = 0; counts[k] = 0; }
    for (int i = 0; i < g_timing.used; ++i) {
        float t = 0.f;
        HIPCHK(hipEventSynchronize(g_timing.ev[2 * i + 1]));
        HIPCHK(hipEventElapsedTime(&t, g_timing.ev[2 * i], g_timing.ev[2 * i + 1]));
        ms[g_timing.phase[i]] += t;
        counts[g_timing.phase[i]] += 1;
    }
    return EELS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ fused batch contraction

struct eels_batch {
    struct Launch {
        int epi, rows, begin, count, tiles;
        int queue = 0;          // its work counter (index after the descriptors in the device table)
    };
    struct Member {
        int plan, batch;
    };
    struct Level {
        std::vector<Member> members;
        std::vector<Launch> g1, g2;
    };
    int precision = 0;
    std::vector<const eels_plan*> plans;
    std::vector<size_t> ws_off;
    std::vector<Level> levels;
    std::vector<GemmDesc> table;
    int n_queues = 0;
    // byte offset of the work counters in the device table (after the descriptors, 256-aligned)
    size_t queue_off() const { return (size_t)round_up((int64_t)std::max<size_t>(table.size(), 1) * sizeof(GemmDesc), 256); }
    size_t queue_bytes() const { return (size_t)round_up((int64_t)std::max(n_queues, 1) * 4, 16); }
};

namespace {

// Bounds of a rebased descriptor's operands, in elements from the arena base, against its
// plan's workspace region [lo, hi) bytes.  rows_a / rows_b: rows read (the probe count when
// rows are gathered through the index list).
bool desc_in_region(const GemmDesc& d, int epi, int64_t rows_a, int64_t rows_b, size_t lo, size_t hi) {
    auto inside = [&](int64_t first, int64_t last_excl, int64_t unit) {
        return first >= 0 && (size_t)(first * unit) >= lo && (size_t)(last_excl * unit) <= hi;
    };
    const int64_t kp = round_up(d.K, 16);
    const int64_t nt1 = std::max(d.n_t, 1) - 1;
    if (!inside(d.a_off, d.a_off + nt1 * d.a_tstride + (rows_a - 1) * d.lda + kp, 8)) return false;
    if (!inside(d.b_off, d.b_off + nt1 * d.b_tstride + (rows_b - 1) * d.ldb + kp, 8)) return false;
    const int64_t np = round_up(d.N_inner, 16);
    if (epi == 0 || epi == 3) return inside(d.c_off, d.c_off + nt1 * d.ldc_t + (int64_t)(d.M - 1) * d.ldc_m + np, 8);
    if (epi == 2) return inside(d.p_off, d.p_off + nt1 * d.ldc_t + (int64_t)(d.M - 1) * d.ldc_m + d.N_inner, 8);
    return inside(d.p_off, d.p_off + (int64_t)(d.tiles_m - 1) * d.ld_part + nt1 * d.N_inner + d.N_inner, 4);
}

}  // namespace

extern "C" {

eels_status eels_batch_create(eels_batch** out, const eels_plan* const* plans, int n_plans, const size_t* ws_offsets,
                              size_t arena_bytes) {
    if (!out || !plans || !ws_offsets || n_plans < 1) {
        set_error("null argument or no plans");
        return EELS_ERR_INVALID_ARG;
    }
    *out = nullptr;
    try {
        auto b = std::make_unique<eels_batch>();
        std::vector<std::pair<size_t, size_t>> regions;
        for (int i = 0; i < n_plans; ++i) {
            if (!plans[i]) {
                set_error("null plan");
                return EELS_ERR_INVALID_ARG;
            }
            const Plan& p = plans[i]->p;
            if (p.precision == EELS_FP32 || (i > 0 && p.precision != b->precision)) {
                set_error("a fused batch needs one split precision for every plan");
                return EELS_ERR_INVALID_ARG;
            }
            if (!p.resident || p.groups.size() > 1) {
                set_error("a fused batch needs plans with resident_s (one slice group)");
                return EELS_ERR_INVALID_ARG;
            }
            if (p.wgram) {
                set_error("a fused batch takes plans of the per-transition detector sum (tuning key 6 = 0)");
                return EELS_ERR_INVALID_ARG;
            }
            if ((ws_offsets[i] & 255) || ws_offsets[i] + p.ws_bytes > arena_bytes) {
                set_error("workspace region misaligned or outside the arena");
                return EELS_ERR_INVALID_ARG;
            }
            b->precision = p.precision;
            b->plans.push_back(plans[i]);
            b->ws_off.push_back(ws_offsets[i]);
            regions.push_back({ws_offsets[i], ws_offsets[i] + p.ws_bytes});
        }
        std::sort(regions.begin(), regions.end());
        for (size_t i = 1; i < regions.size(); ++i)
            if (regions[i].first < regions[i - 1].second) {
                set_error("workspace regions overlap");
                return EELS_ERR_INVALID_ARG;
            }
        // each plan's batches in its execute order (slices descending)
        std::vector<std::vector<int>> seq(n_plans);
        size_t n_levels = 0;
        for (int i = 0; i < n_plans; ++i) {
            const Plan& p = b->plans[i]->p;
            for (int j = p.nz - 1; j >= 0; --j)
                if (p.slices[j].ion)
                    for (int bi : p.slices[j].batches) seq[i].push_back(bi);
            n_levels = std::max(n_levels, seq[i].size());
        }
        for (size_t k = 0; k < n_levels; ++k) {
            eels_batch::Level lv;
            // descriptors per launch group (epilogue, rows), in member order
            std::vector<std::vector<GemmDesc>> d1, d2;
            auto group = [](std::vector<eels_batch::Launch>& g, std::vector<std::vector<GemmDesc>>& dv, int epi,
                             int rows) -> int {
                for (size_t q = 0; q < g.size(); ++q)
                    if (g[q].epi == epi && g[q].rows == rows) return (int)q;
                g.push_back({epi, rows, 0, 0, 0});
                dv.emplace_back();
                return (int)g.size() - 1;
            };
            for (int i = 0; i < n_plans; ++i) {
                if (k >= seq[i].size()) continue;
                const Plan& p = b->plans[i]->p;
                const Batch& bt = p.batches[seq[i][k]];
                lv.members.push_back({i, seq[i][k]});
                // the device bases of this plan's launches, as byte offsets from the arena
                const Dev hd = make_dev(p, (void*)(uintptr_t)b->ws_off[i]);
                const size_t lo = b->ws_off[i], hi = b->ws_off[i] + p.ws_bytes;
                const int64_t blob_i = (int64_t)((uintptr_t)hd.blob / 4);
                for (int gemm = 1; gemm <= 2; ++gemm) {
                    const SplitCall c = gemm == 1 ? split_gemm1(p, hd) : split_gemm2(p, hd);
                    const int rows = gemm == 1 ? bt.d1_rows : bt.d2_rows;
                    const int q = gemm == 1 ? group(lv.g1, d1, c.epi, rows) : group(lv.g2, d2, c.epi, rows);
                    std::vector<GemmDesc>& dst = gemm == 1 ? d1[q] : d2[q];
                    eels_batch::Launch& L = gemm == 1 ? lv.g1[q] : lv.g2[q];
                    const int begin = gemm == 1 ? bt.d1_begin : bt.d2_begin;
                    const int count = gemm == 1 ? bt.d1_count : bt.d2_count;
                    for (int e = 0; e < count; ++e) {
                        GemmDesc d = p.descs[begin + e];
                        if (d.h_off >= 0) {
                            set_error("fused batch: descriptor with an H prologue");
                            return EELS_ERR_INTERNAL;
                        }
                        const bool gather_a = d.idx_off >= 0 && (d.flags & GD_IDX_A);
                        const bool gather_b = d.idx_off >= 0 && !(d.flags & GD_IDX_A);
                        d.a_off += (int64_t)((uintptr_t)c.A / 8);
                        d.b_off += (int64_t)((uintptr_t)c.B / 8);
                        if (c.epi == 0 || c.epi == 3) d.c_off += (int64_t)((uintptr_t)c.C / 8);
                        else if (c.epi == 2) d.p_off += (int64_t)((uintptr_t)c.P / 8);
                        else d.p_off += (int64_t)((uintptr_t)c.P / 4);
                        if (d.idx_off >= 0) d.idx_off += blob_i;
                        if (!desc_in_region(d, c.epi, gather_a ? p.P : d.M, gather_b ? p.P : d.N_inner, lo, hi)) {
                            set_error("fused batch: a merged descriptor leaves its plan's workspace");
                            return EELS_ERR_INTERNAL;
                        }
                        if (d.idx_off >= 0 &&
                            (size_t)(d.idx_off + (gather_a ? d.M : d.N_inner)) * 4 > lo + p.off_blob + p.blob.size() * 4) {
                            set_error("fused batch: an index list leaves its plan's table");
                            return EELS_ERR_INTERNAL;
                        }
                        d.tile_start = L.tiles;
                        L.tiles += d.tiles_m * d.tiles_n * d.n_t;
                        dst.push_back(d);
                    }
                }
            }
            for (int gemm = 1; gemm <= 2; ++gemm) {
                auto& g = gemm == 1 ? lv.g1 : lv.g2;
                auto& dv = gemm == 1 ? d1 : d2;
                for (size_t q = 0; q < g.size(); ++q) {
                    g[q].begin = (int)b->table.size();
                    g[q].count = (int)dv[q].size();
                    g[q].queue = b->n_queues++;
                    b->table.insert(b->table.end(), dv[q].begin(), dv[q].end());
                }
            }
            b->levels.push_back(std::move(lv));
        }
        *out = b.release();
        return EELS_OK;
    } catch (const std::exception& e) {
        set_error(e.what());
        return EELS_ERR_INTERNAL;
    }
}

eels_status eels_batch_table_bytes(const eels_batch* b, size_t* bytes) {
    if (!b || !bytes) return EELS_ERR_INVALID_ARG;
    *bytes = b->queue_off() + b->queue_bytes();
    return EELS_OK;
}

eels_status eels_batch_upload(const eels_batch* b, void* d_table, void* stream) {
    if (!b || !d_table || ((uintptr_t)d_table & 255)) {
        set_error("null batch or table, or table not 256-byte aligned");
        return EELS_ERR_INVALID_ARG;
    }
    if (!b->table.empty())
        HIPCHK(hipMemcpyAsync(d_table, b->table.data(), b->table.size() * sizeof(GemmDesc), hipMemcpyHostToDevice,
                              (hipStream_t)stream));
    return EELS_OK;
}

eels_status eels_batch_contract(const eels_batch* b, void* d_arena, const void* d_table, const void* const* d_H,
                                double* const* d_maps, void* stream) {
    if (!b || !d_arena || !d_table || !d_maps || ((uintptr_t)d_arena & 255)) {
        set_error("null argument or arena not 256-byte aligned");
        return EELS_ERR_INVALID_ARG;
    }
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
        if (!d_maps[i] || (b->plans[i]->p.n_trans_total > 0 && (!d_H || !d_H[i]))) {
            set_error("null map or transition potentials");
            return EELS_ERR_INVALID_ARG;
        }
    hipStream_t st = (hipStream_t)stream;
    char* arena = (char*)d_arena;
    const GemmDesc* table = (const GemmDesc*)d_table;
    // the grouped GEMMs run persistently: each launch's resident workgroups take tiles from its
    // work counter, zeroed here by a kernel (so that a captured graph resets them on every replay)
    int* queues = (int*)((char*)const_cast<void*>(d_table) + b->queue_off());
    std::vector<Dev> devs;
    for (int i = 0; i < n; ++i) devs.push_back(make_dev(b->plans[i]->p, arena + b->ws_off[i]));
    const int nst = tune_get(TUNE_SC_STAGES);
    g_timing.used = 0;
    launch_fill_zero(queues, b->queue_bytes(), st);
    for (const auto& lv : b->levels) {
        for (const auto& m : lv.members) {
            const Plan& p = b->plans[m.plan]->p;
            producers_before_gemm1(p, devs[m.plan], (const float2*)d_H[m.plan], p.batches[m.batch], st);
        }
        {
            TimeScope ts(EELS_PHASE_GEMM1, st);
            for (const auto& g : lv.g1)
                launch_cgemm_sc(b->precision, g.epi, nst, table + g.begin, g.count, g.tiles, arena, arena, arena,
                                (float*)arena, (const int*)arena, st, g.rows, queues + g.queue);
        }
        for (const auto& m : lv.members) {
            const Plan& p = b->plans[m.plan]->p;
            producers_after_gemm1(p, devs[m.plan], (const float2*)d_H[m.plan], p.batches[m.batch], st);
        }
        {
            TimeScope ts(EELS_PHASE_GEMM2, st);
            for (const auto& g : lv.g2)
                launch_cgemm_sc(b->precision, g.epi, nst, table + g.begin, g.count, g.tiles, arena, arena, arena,
                                (float*)arena, (const int*)arena, st, g.rows, queues + g.queue);
        }
        for (const auto& m : lv.members) {
            const Plan& p = b->plans[m.plan]->p;
            reduce_batch(p, devs[m.plan], d_maps[m.plan], p.batches[m.batch], st);
        }
    }
    for (int i = 0; i < n; ++i) finish_map(b->plans[i]->p, devs[i], d_maps[i], st);
    HIPCHK(hipGetLastError());
    return EELS_OK;
}

eels_status eels_batch_destroy(eels_batch* b) {
    delete b;
    return EELS_OK;
}

}  // extern "C"
