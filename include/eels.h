/*
 * eels.h -- C ABI of the MI355X PRISM STEM-EELS library (libeels.so).
 *
 * The library computes an atomic-resolution STEM-EELS map with the linear-scaling
 * scattering-matrix method of Brown, Ciston and Ophus (arXiv:1908.07628):
 *
 *   S_1(j)  plane waves of the probe-forming aperture multisliced to the entrance of
 *           slice j (Sec. 3, PRISM STEM-EELS algorithm; Eq. MSop for one slice);
 *   S_2(j)  the transposed scattering matrix that takes a wave present at the entrance
 *           of slice j to the detector beams at the exit (Eq. MSTop, exact transpose);
 *   A_n(q,R) = sum_r S_2(j)[q](r) H_n(r) sum_k c_k(R) S_1(j)[k](r)   (Eqs. Hn0Psi, SHn0)
 *   I(R)    = f^2 sum_{sites, n, q} |A_n(q,R)|^2                     (map accumulation)
 *
 * with c_k(R) = s A(k) exp(-i chi(k)) exp(-2 pi i k.R) the probe coefficients (Eq. illum),
 * T_j = exp(i sigma V_j) and P_j = B(k) exp(-i pi lambda dz_j k^2) (Eq. MSop), B the
 * circular band limit.  The transition of a slice acts at its entrance, before T_j.
 *
 * Conventions
 *   - Arrays are row-major [y][x] (x fastest).  Complex values are interleaved
 *     (re, im) single-precision pairs ("complex64").
 *   - Forward transforms carry exp(-2 pi i r.g) (footnote to Eq. 4).
 *   - Every function returns an eels_status; no C++ exception crosses the ABI.
 *   - The library never frees caller memory.  Device buffers passed to eels_execute
 *     are owned by the caller and must stay valid until the stream has finished.
 *   - A plan is immutable after creation and may be used for several concurrent
 *     executions on different streams with different workspaces.
 */
#ifndef EELS_H
#define EELS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EELS_VERSION_MAJOR 0
#define EELS_VERSION_MINOR 4

typedef int eels_status;
enum {
    EELS_OK = 0,
    EELS_ERR_INVALID_ARG = 1,      /* a size, pointer or parameter is out of range       */
    EELS_ERR_BANDLIMIT = 2,        /* an aperture or detector beam lies outside the band  */
    EELS_ERR_UNSUPPORTED_SIZE = 3, /* grid side not a power of two in [16, 1024] or 384  */
    EELS_ERR_WORKSPACE = 4,        /* workspace pointer null or smaller than required     */
    EELS_ERR_OOM = 5,              /* the problem does not fit the memory budget          */
    EELS_ERR_DEVICE = 6,           /* a HIP call failed (message via eels_last_error)     */
    EELS_ERR_CANCELLED = 7,        /* a queued request was cancelled                      */
    EELS_ERR_INTERNAL = 8
};

enum { EELS_FP32 = 0, EELS_BF16_SPLIT = 1, EELS_FP16_SPLIT = 2 };
enum { EELS_ORDER_AUTO = 0, EELS_ORDER_S_FIRST = 1, EELS_ORDER_PROBE_FIRST = 2 };

/* One ionised atom: its transitions act at the entrance of `slice` (0-based).
 * H rows h_offset .. h_offset + n_trans - 1 hold its transition potentials. */
typedef struct {
    int slice;
    int n_trans;
    double x_A, y_A;
    int64_t h_offset;
} eels_site;

/* The problem statement (all host values; the library copies what it keeps).
 *
 * Grid and cell: nx x ny pixels over lx x ly Angstrom (periodic).  Slices: n_slices
 * thicknesses dz_A[].  Beam: energy_eV; lambda_A and sigma (rad/(V*A)) override the
 * relativistic values when > 0.  Probe: aperture semi-angle, optional defocus and Cs
 * (Angstrom) in chi(k) = pi lambda k^2 (Cs lambda^2 k^2 / 2 - defocus).  Detector:
 * inner/outer semi-angles (inclusive).  interp_f: PRISM interpolation factor (beams on
 * the lattice f Z^2 / L).  bandlimit: fraction of Nyquist of the circular band limit
 * (0 -> 2/3).  window_A: side of the crop window of the contraction (Sec. 4.B);
 * 0 -> full cell.  Probes: n_probes (x, y) positions in Angstrom.  Sites: n_sites
 * entries; n_trans_total rows of H.  max_workspace_bytes: memory budget for the plan's
 * workspace (0 -> unlimited); slices are processed in groups to stay within it.
 * Full-cell windows are contracted in the basis of band-limited plane waves: because
 * S_2(j)[q] = T_j fft2(P_j x) with P_j zero outside the band, sum_r S_2 H S_1 equals
 * sum over band pixels g of (P_j x)(g) fft2(T_j H S_1)(g), about 1/3 of the pixels. */
typedef struct {
    int nx, ny;
    double lx_A, ly_A;
    int n_slices;
    const double* dz_A;
    double energy_eV;
    double lambda_A;
    double sigma;
    double aperture_mrad;
    double det_inner_mrad, det_outer_mrad;
    double defocus_A, cs_A;
    int interp_f;
    double bandlimit;
    double window_A;
    int n_probes;
    const double* probe_xy;
    int n_sites;
    const eels_site* sites;
    int64_t n_trans_total;
    int precision;
    int order;
    size_t max_workspace_bytes;
    int real_space;          /* 1: contract full-cell windows pixel by pixel instead of in the
                                band basis (same result, about 3x more GEMM work)            */
    int resident_s;          /* 1: keep the S_2 capture of every ionised slice in the workspace
                                (needs one slice group), so that a later eels_execute_ex with
                                EELS_EXEC_SKIP_SWEEPS can reuse the S-matrices              */
    int detector_sum;        /* EELS_DETSUM_*: how sum_{n,q} |A_n(q,R)|^2 is formed (order S)  */
    int s1_mode;             /* EELS_S1_STORED (exact), EELS_S1_INVERSE or EELS_S2_RETREAT
                                (the inverse multislice of Sec. 4.C on S_1 or on S_2)         */
    int n_images;            /* elastic companion images (0 .. EELS_MAX_IMAGES), interp_f = 1  */
    const double* image_detectors_mrad;  /* [n_images][2] inner, outer semi-angle (inclusive);
                                outer <= 0 means the band limit                              */
} eels_problem;

/* Elastic companion images (the incoherent bright-field and annular dark-field images shown
 * beside the EELS map in the Results' nanoparticle discussion, which also divides the EELS
 * map by the iBF image with the EELS detector's angles).  Image d is
 *     I_d(R) = sum_{q in D_d} |psi_exit(q, R)|^2,  psi_exit(., R) = sum_k c_k(R) S_1^exit[k],
 * the elastic exit wave of probe R on the pixels of the ring D_d, as a fraction of the
 * incident beam.  With interp_f = 1 it equals c(R)^H G_d c(R), G_d = S_d^H S_d over the
 * ring's pixels, which is how it is computed (FP32 Gram GEMM, FP64 quadratic form). */
enum { EELS_MAX_IMAGES = 8 };

/* Detector sum of the S-first order.  DIRECT: A_n(q, R) = sum_k Z_n(q, k) c_k(R) by a second
 * GEMM per transition with |.|^2 summed over q in its epilogue.  GRAM: with every probe
 * covering every site (interp_f = 1), sum_{n,q} |A_n(q,R)|^2 = c(R)^H G c(R) with the
 * Hermitian G = sum_n Z_n^H Z_n (N_1 x N_1, accumulated in FP64); the second GEMM forms
 * the upper-triangle tiles of each site's Z^H Z and one FP64 quadratic form per probe
 * finishes the map (about 5x fewer flops than DIRECT for the crystal maps).  AUTO picks
 * GRAM where it applies (order S, interp_f = 1, band basis or split precision). */
enum { EELS_DETSUM_AUTO = 0, EELS_DETSUM_DIRECT = 1, EELS_DETSUM_GRAM = 2 };

/* How S_1 reaches the ionised slices.  STORED: the forward sweep captures S_1 at every
 * ionised slice on the way down and keeps the windows until the transposed S_2 sweep
 * reaches them (exact; slice groups bound the memory).  INVERSE: the inverse multislice of
 * Sec. 4.C, Eq. MSinvop: S_1 is swept to the exit plane and then retreated slice by slice
 * with M_j^-1 = F conj(T_j) F^-1 conj(P_j) in step with the S_2 sweep, so only one slice's
 * windows are ever held.  Approximate: intensity that multislice pushed beyond the band
 * limit is not recovered.  Not combinable with resident_s. */
/* EELS_S1_STORED: S_1 windows of the ionised slices stored by the forward sweep, S_2 by one
 * exact transposed sweep (exact).  EELS_S1_INVERSE: S_1 multisliced to the exit and retreated
 * slice by slice with the inverse multislice (Eq. MSinvop) beside the transposed sweep.
 * EELS_S2_RETREAT: as Sec. 4.C describes it, S_2 formed for the entrance by the transposed sweep
 * and retreated towards the exit with the inverse of each transposed step, beside the forward
 * S_1 sweep.  Both inverse modes keep one slice's windows and are approximate where intensity
 * left the band limit.  EELS_S2_RETREAT plans contract in real space (real_space implied). */
enum { EELS_S1_STORED = 0, EELS_S1_INVERSE = 1, EELS_S2_RETREAT = 2 };

/* Derived sizes of a plan (filled by eels_plan_info). */
typedef struct {
    int n_beams_in;          /* N_1: aperture beams on the f-lattice                      */
    int n_beams_out;         /* N_2: detector beams on the f-lattice                      */
    int n_beams_in_fine;     /* aperture beams at f = 1 (probe normalisation)             */
    int n_live_x;            /* kx columns inside the band limit                          */
    int window_nx, window_ny;/* crop window side in pixels (nx, ny if full cell)          */
    int k_pixels;            /* pixels per window                                         */
    int k_stride;            /* padded window stride (complex elements)                  */
    int n_ion_slices;        /* slices that hold at least one site                        */
    int n_groups;            /* slice groups (forward sweep repeated once per group)      */
    int n_batches;           /* contraction batches                                       */
    int order;               /* EELS_ORDER_S_FIRST or EELS_ORDER_PROBE_FIRST              */
    int band_basis;          /* 1 if full-cell windows are contracted in the band basis    */
    int band_pixels;         /* pixels inside the circular band limit                      */
    double lambda_A, sigma;
    double gemm_flops;       /* useful complex-GEMM flops (8 M N K summed)                */
    double sweep_bytes;      /* algorithmic HBM bytes of the two sweeps                   */
    double sweep_beam_slices;/* beam-slice passes of the two sweeps                       */
    size_t workspace_bytes;
    int gram_form;           /* 1 if the detector sum uses the Gram form (EELS_DETSUM_GRAM) */
    int window_gram_form;    /* 1 if order P uses the window-Gram detector sum (tuning key 6) */
    int raster_form;         /* DFT side M of its raster form (tuning key 7), 0 if not used  */
    int n_checkpoints;       /* S_1 states kept for later slice groups (tuning key 8)      */
} eels_plan_info;

typedef struct eels_plan eels_plan;

eels_status eels_get_version(int* major, int* minor);
const char* eels_status_string(eels_status s);
/* Text of the last error on the calling thread (empty if none). */
const char* eels_last_error(void);

/* Host only: validates the problem, builds beam lists (ordered by lattice row, then
 * column), crop windows, probe eligibility, the contraction order and the workspace
 * layout.  Touches no device.  Errors: INVALID_ARG, BANDLIMIT, UNSUPPORTED_SIZE, OOM. */
eels_status eels_plan_create(eels_plan** out, const eels_problem* prob);
eels_status eels_plan_workspace_bytes(const eels_plan* p, size_t* bytes);
eels_status eels_plan_info_get(const eels_plan* p, eels_plan_info* info);
/* Lattice coordinates (a, b) of the aperture (which = 0) or detector (which = 1)
 * beams, k = (f a / lx, f b / ly); ab must hold 2 * count ints. */
eels_status eels_plan_beams(const eels_plan* p, int which, int* ab, int count);
eels_status eels_plan_destroy(eels_plan* p);

/* Device: computes the map.  d_V: float32 [n_slices][ny][nx] projected potential
 * (V*A).  d_H: complex64 [n_trans_total][wy][wx] transition potentials on each site's
 * window (window pixel (u, v) is grid pixel (ix0 - h + u, iy0 - h + v) mod n, ix0 the
 * site's nearest pixel), or [n_trans_total][ny][nx] on the full grid.  d_map: float64
 * [n_probes], overwritten.  d_workspace: at least eels_plan_workspace_bytes bytes,
 * 256-byte aligned.  All work is enqueued on `stream` (a hipStream_t, 0 = default);
 * no device memory is allocated and the host does not wait for the device. */
eels_status eels_execute(const eels_plan* p, const float* d_V, const void* d_H, double* d_map,
                         void* d_workspace, size_t workspace_bytes, void* stream);

/* eels_execute with options.  flags:
 *   EELS_EXEC_SKIP_UPLOAD  the plan's tables are already in this workspace (uploaded by an
 *                          earlier execute of the same plan on it): enqueue kernels only, so
 *                          the call can be captured into a HIP graph.
 *   EELS_EXEC_SKIP_SWEEPS  reuse the S-matrix data (S_1 windows and every slice's S_2
 *                          capture) left in the workspace by an earlier execute of a plan
 *                          with the same S signature (eels_plan_s_signature) on the same V
 *                          and H; needs resident_s.  Only the set-up and the contractions run,
 *                          e.g. for a new set of probe positions.
 *   EELS_EXEC_SWEEPS_ONLY  the set-up and both sweeps only (every S_1 window and every
 *                          slice's S_2 capture left in the workspace, d_map zeroed); the
 *                          contractions follow in eels_batch_contract.  Needs resident_s.
 * Errors as eels_execute; INVALID_ARG for SKIP_SWEEPS or SWEEPS_ONLY without resident_s, or
 * both together. */
enum { EELS_EXEC_SKIP_UPLOAD = 1, EELS_EXEC_SKIP_SWEEPS = 2, EELS_EXEC_SWEEPS_ONLY = 4 };
eels_status eels_execute_ex(const eels_plan* p, const float* d_V, const void* d_H, double* d_map,
                            void* d_workspace, size_t workspace_bytes, void* stream, unsigned flags);

/* eels_execute without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid allocation).  The
 * workspace is a fixed 128 MiB device array inside the library (one per device, held until the
 * process ends); the call allocates nothing and enqueues on `stream` like eels_execute.  Plans
 * whose eels_plan_workspace_bytes exceed 128 MiB (about the size of the 64 x 64-pixel cells
 * with a few hundred beams) are refused with EELS_ERR_WORKSPACE.  Every call on one device
 * shares that array, so calls that overlap on one device (different streams or threads
 * without ordering) race: order them on one stream or serialise them.  The map equals that of
 * eels_execute bit for bit.  Errors as eels_execute. */
eels_status eels_execute_noalloc(const eels_plan* p, const float* d_V, const void* d_H, double* d_map, void* stream);

/* As eels_execute_ex, and also writes the plan's elastic companion images:
 * d_images float64 [n_images][n_probes], overwritten (may be null when n_images = 0).  The
 * forward sweep then continues to the exit plane and captures the exit wave's band
 * coefficients.  With EELS_EXEC_SKIP_SWEEPS the forward sweep is rerun for the images (the
 * S_2 data stay resident).  Errors as eels_execute_ex. */
eels_status eels_execute_images(const eels_plan* p, const float* d_V, const void* d_H, double* d_map, double* d_images,
                                void* d_workspace, size_t workspace_bytes, void* stream, unsigned flags);

/* 64-bit signature of everything the S-matrix data in a workspace depends on (geometry,
 * slices, optics, beam lattices, windows, sites, storage format and the workspace
 * offsets of the S data), but not of the probes.  Equal signatures (with equal V and H)
 * mean the S data of one plan's execute serve the other. */
eels_status eels_plan_s_signature(const eels_plan* p, uint64_t* sig);

/* Fused contraction of a batch of maps (many specimens of uneven size).  Each map's
 * contraction is the per-site sum of Eq. SHn0 (Sec. 3, second algorithm); the plans'
 * site batches are taken level by level (the k-th batch of every plan in its execute
 * order), and each level's first and second GEMMs of all plans run as one grouped launch
 * per kernel variant over a merged descriptor table, so that small specimens share the
 * matrix cores instead of launching one small grid each.
 * Plans: split precision (all the same), resident_s, one slice group, the per-transition
 * detector sum (made with tuning key 6 = 0, or where the window-Gram form does not apply).
 * Workspaces are regions of one caller-owned arena: plan i at d_arena + ws_offsets[i]
 * (256-byte aligned, eels_plan_workspace_bytes long, not overlapping, within arena_bytes).
 *   eels_batch_create   host only: checks the plans, builds and bounds-checks the merged
 *                       descriptors (their offsets count from the arena base).  The plans
 *                       must outlive the batch.
 *   eels_batch_table_bytes  device bytes of the merged table (the descriptors and one work
 *                       counter per grouped launch).
 *   eels_batch_upload   copies the table to d_table (256-byte aligned, caller-owned) on
 *                       `stream`; once, before any (captured) contraction.
 *   eels_batch_contract enqueues on `stream`, after every plan's eels_execute_ex with
 *                       EELS_EXEC_SWEEPS_ONLY on its workspace has completed (or precedes
 *                       it on the stream): the producers per plan, the grouped GEMMs per
 *                       level, the FP64 reductions into d_maps[i] (float64 [n_probes of plan
 *                       i], zeroed by the sweeps-only execute).  d_H[i]: plan i's transition
 *                       potentials.  No allocation, no host synchronisation (capturable).
 *                       Each grouped GEMM runs as a persistent launch: the device's resident
 *                       workgroups take (plan, site, tile) work items from that launch's
 *                       counter in d_table, which the call first zeroes with a kernel (so
 *                       every replay of a captured graph starts from zero; calls sharing one
 *                       d_table must not overlap).
 * Results equal each plan's own eels_execute bit for bit.  Errors: INVALID_ARG (null
 * pointers, mixed or FP32 precision, non-resident or window-Gram plans, workspace
 * regions), INTERNAL (a merged descriptor outside its plan's workspace), DEVICE. */
typedef struct eels_batch eels_batch;
eels_status eels_batch_create(eels_batch** out, const eels_plan* const* plans, int n_plans, const size_t* ws_offsets,
                              size_t arena_bytes);
eels_status eels_batch_table_bytes(const eels_batch* b, size_t* bytes);
eels_status eels_batch_upload(const eels_batch* b, void* d_table, void* stream);
eels_status eels_batch_contract(const eels_batch* b, void* d_arena, const void* d_table, const void* const* d_H,
                                double* const* d_maps, void* stream);
eels_status eels_batch_destroy(eels_batch* b);

/* Conventional multislice STEM-EELS (Sec. 3, first algorithm) on the same GPU, for comparing
 * the two algorithms on equal hardware.  For every probe the elastic wave is multisliced;
 * at the entrance of every ionised slice each transition n of each site spawns the inelastic
 * wave H_n psi, which is multisliced to the exit plane and summed as |.|^2 over the detector
 * beams.  Probes are processed probe_chunk at a time (all their inelastic waves at once).
 * FP32 waves, FP64 map written to d_map [n_probes] (overwritten).  Needs interp_f = 1;
 * windowed transition potentials are placed into full planes first.  d_workspace: 256-byte
 * aligned, at least eels_conventional_workspace_bytes(p, probe_chunk) bytes (its own layout:
 * tables, T_j, P_j, and for one chunk the entrance waves, (1 + n_trans) waves per probe of
 * ny * ldx complex64 and their exit band coefficients), caller-owned; 0 is returned for
 * probe_chunk < 1.  Errors: INVALID_ARG for null pointers, probe_chunk < 1 or interp_f > 1,
 * WORKSPACE for a small or misaligned workspace, DEVICE for a failed launch. */
size_t eels_conventional_workspace_bytes(const eels_plan* p, int probe_chunk);
eels_status eels_conventional_map(const eels_plan* p, const float* d_V, const void* d_H, double* d_map,
                                  int probe_chunk, void* d_workspace, size_t workspace_bytes, void* stream);

/* Diagnostics (same workspace contract).  Write the real-space rows of S_1(j)
 * (scaled by nx*ny, i.e. unit-modulus plane waves at j = 0) as complex64
 * [N_1][ny][nx], or of S_2(j) as complex64 [N_2][ny][nx]. */
eels_status eels_debug_s1(const eels_plan* p, const float* d_V, int slice, void* d_out,
                          void* d_workspace, size_t workspace_bytes, void* stream);
eels_status eels_debug_s2(const eels_plan* p, const float* d_V, int slice, void* d_out,
                          void* d_workspace, size_t workspace_bytes, void* stream);

/* Diagnostic complex GEMM through the same kernels as the contraction:
 * C[m][n] = sum_k A[m][k] * B[n][k] (no conjugation), complex64, row-major with
 * leading dimensions lda, ldb, ldc (complex elements; lda and ldb even).  If d_norm2 is
 * not null, d_norm2[n] = sum_m |C[m][n]|^2 (float64) is written instead of C.
 * precision: EELS_FP32 / EELS_BF16_SPLIT / EELS_FP16_SPLIT (split operands are converted
 * to the split-complex storage first).  d_work: at least eels_gemm_work_bytes(m, n, k)
 * bytes, 256-byte aligned.  Synchronises `stream` before returning. */
size_t eels_gemm_work_bytes(int m, int n, int k);
eels_status eels_debug_cgemm(int precision, int m, int n, int k, const void* d_A, int lda,
                             const void* d_B, int ldb, void* d_C, int ldc, double* d_norm2,
                             void* d_work, void* stream);

/* Map arithmetic on device maps (float64, caller-owned, enqueued on `stream`).
 *   eels_map_mean   d_out[i] = (1 / n_maps) sum_c d_maps[c * n + i], summed in configuration
 *                   order c = 0 .. n_maps-1 in FP64: the frozen-phonon map, the average of the
 *                   maps of n_maps thermal configurations (the Results' nanoparticle run is one
 *                   frozen-phonon pass; more passes are averaged).  d_out may alias no input.
 *   eels_map_ratio  d_out[i] = d_num[i] / d_den[i] where d_den[i] > 0, else 0: the BF-corrected
 *                   map, the EELS map divided by the incoherent bright-field image of the EELS
 *                   detector's angles (Results, nanoparticle discussion).  d_out may be d_num.
 * Errors: INVALID_ARG for null pointers, n_maps < 1 or n < 0; DEVICE for a failed launch. */
eels_status eels_map_mean(double* d_out, const double* d_maps, int n_maps, int64_t n, void* stream);
eels_status eels_map_ratio(double* d_out, const double* d_num, const double* d_den, int64_t n, void* stream);

/* Serving: EELS-map requests solved as they arrive on one GPU (continuous batching).  The
 * problem statement of each request is that of eels_plan_create (Sec. 3: specimen slices,
 * transition potentials, probe positions, aperture and detector angles in, map out).
 *
 *   eels_server_create   starts a dispatcher thread on `device` with `max_slots` streams (1 to
 *                        64) and an HBM budget for the workspaces it allocates (the caller's
 *                        inputs and maps are not counted).
 *   eels_server_submit   plans the request on the calling thread (resident_s forced, one slice
 *                        group) and queues it.  d_V, d_H: the request's device inputs as for
 *                        eels_execute, already written (the server hashes their content at
 *                        submit); d_map: float64 [n_probes], written when the request is done.
 *                        All three stay caller-owned and must stay valid until the request is
 *                        done.  *ticket identifies the request.  Errors: those of
 *                        eels_plan_create, OOM when the workspace exceeds the whole budget.
 *   Admission           first fit in arrival order while a slot is free and the workspace fits
 *                        the budget (idle resident workspaces are freed least recently used to
 *                        make room); a request overtaken 4 times blocks the ones behind it
 *                        until it fits.  Admitted requests run concurrently on their streams.
 *   Residency           a finished request's workspace stays allocated (its S-matrix data),
 *                        keyed by the content of V and H and the plan's S signature; a later
 *                        request with the same key runs with EELS_EXEC_SKIP_SWEEPS on it.
 *   eels_server_poll     *done = 1 once the request has finished (its map written) or ended with
 *                        an error; `t` (may be null) receives its timing and status.
 *   eels_server_wait     as poll, waiting up to timeout_s seconds for the request to finish.
 *   eels_server_cancel   ends a queued request with EELS_ERR_CANCELLED; INVALID_ARG if it has
 *                        started or finished.
 *   eels_server_release  forgets a finished request's record (its ticket becomes invalid).
 *   eels_server_get_stats  counters since creation and the memory the server holds.
 *   eels_server_destroy  cancels queued requests, waits for running ones, frees every
 *                        workspace and stops the thread.
 * A request's map equals that of a lone eels_execute of the same problem bit for bit, alone
 * and in any mix (same kernels in the same order, no atomics).  Failures of one request (a
 * failed allocation, a launch error) end that request with its status and release its slot
 * and memory.  The server's functions are thread-safe; destroy must not race other calls. */
typedef struct eels_server eels_server;
typedef struct {
    double arrival_s, start_s, finish_s;   /* seconds since eels_server_create (steady clock)  */
    int resident_hit;                      /* 1: ran on a resident workspace (sweeps skipped)   */
    eels_status status;                    /* EELS_OK, or the error that ended the request      */
    size_t workspace_bytes;                /* the request's footprint                           */
} eels_request_timing;
typedef struct {
    int64_t submitted, completed, failed, cancelled, resident_hits, evictions;
    size_t resident_bytes;                 /* workspaces kept for residency                     */
    int64_t resident_entries;
    size_t running_bytes;                  /* fresh workspaces of running requests              */
} eels_server_stats;
eels_status eels_server_create(eels_server** out, int device, size_t hbm_budget_bytes, int max_slots);
eels_status eels_server_submit(eels_server* s, const eels_problem* prob, const float* d_V, const void* d_H,
                               double* d_map, uint64_t* ticket);
eels_status eels_server_poll(eels_server* s, uint64_t ticket, int* done, eels_request_timing* t);
eels_status eels_server_wait(eels_server* s, uint64_t ticket, double timeout_s, int* done, eels_request_timing* t);
eels_status eels_server_cancel(eels_server* s, uint64_t ticket);
eels_status eels_server_release(eels_server* s, uint64_t ticket);
eels_status eels_server_get_stats(eels_server* s, eels_server_stats* out);
eels_status eels_server_destroy(eels_server* s);

/* The server's admission policy on its own (host only, for schedulers and tests): requests
 * (ticket, footprint, arrival) are offered in arrival order; eels_admission_admit returns up to
 * max_out tickets to start now (first fit while fewer than max_slots run and used + footprint
 * <= capacity; once the oldest queued request has been overtaken max_overtake times nothing
 * behind it is admitted until it fits); finish releases a running ticket's footprint.  offer
 * returns OOM for a footprint above the budget; cancel INVALID_ARG for a ticket not queued. */
typedef struct eels_admission eels_admission;
eels_status eels_admission_create(eels_admission** out, size_t budget_bytes, int max_slots, int max_overtake);
eels_status eels_admission_offer(eels_admission* a, uint64_t ticket, size_t footprint, double arrival);
int eels_admission_admit(eels_admission* a, size_t capacity, uint64_t* tickets, int max_out);
eels_status eels_admission_finish(eels_admission* a, uint64_t ticket);
eels_status eels_admission_cancel(eels_admission* a, uint64_t ticket);
size_t eels_admission_used(const eels_admission* a);
eels_status eels_admission_destroy(eels_admission* a);

/* Process-wide kernel tuning knobs, read at launch time (keys 3 to 7: at plan time; the
 * autotuner sets keys 0, 1, 4 and 5).
 * key 0: LDS pipeline of the split-precision GEMM: 2 (two stages of 16-complex tiles, two
 *        workgroups per CU, default), 3 (three such stages, one workgroup per CU), 4 or 5
 *        (four or five stages of 8-complex tiles, two workgroups per CU).
 * key 1: tile order of the contraction GEMMs within a problem: 0 m-fastest (the workgroups
 *        in flight share B tiles), 1 n-fastest (they share A tiles), 2 XCD-aware (default;
 *        each of the 8 XCDs takes one contiguous range of tiles in groups of 8 m tiles, so
 *        the workgroups sharing one L2 cover a compact patch of the output).
 * key 2: instruction schedule of the two-stage split GEMM: bit 0 reads the next 8-complex
 *        step's operand fragments from LDS before the current step's MFMAs, bit 1 raises
 *        the wave's issue priority while it issues MFMAs (0 default).
 * key 3: rows of the Gram form's first GEMM: 1 (default) the transitions of a site stacked
 *        into one M = n_t N_1, 0 one N_1-row problem per transition.
 * key 4: tiles of the first contraction GEMM in split precision (both orders): 1 (default)
 *        256 x 128 tiles of 8 waves, one workgroup per CU; 0 128 x 128 tiles of 4 waves.
 * key 5: tiles of the second contraction GEMM in split precision with the per-probe
 *        detector sum (not the Gram form): 1 (default) 256 x 128 tiles of 8 waves; 0
 *        128 x 128 tiles of 4 waves.
 * key 6: detector sum of order P with cropped windows, in every precision (Sec. 3 second
 *        algorithm, Eq. SHn0): 1 the window-Gram form.  Per site, M = S_2w^H S_2w over the
 *        detector beams (K x K window pixels, one Gram GEMM for all transitions), G = M o
 *        sum_t conj(H_t) H_t^T, and I(R) = f^2 Psi_R^H G Psi_R (one GEMM G Psi and a
 *        per-probe dot product) instead of n_t products (S_2w o H_t) Psi.  Used when the
 *        window has at most 4096 pixels and the form needs fewer flops over the plan's
 *        sites (it does with many eligible probes per site): 1 (default) this form where
 *        it needs fewer flops, 2 wherever it applies, 0 never (the per-transition
 *        products).  A fused batch (eels_batch_create) takes plans made with 0.
 * key 7: the raster form of the window-Gram detector sum.  When every probe lies on a raster
 *        aligned with the beam lattice, R = R_0 + (i L_x / (f M), j L_y / (f M)) with integer i, j
 *        and M = 64 (e.g. a 256 x 256 scan at f = 4), and the aperture beams' lattice coordinates
 *        (a, b) each span fewer than M values, c_k(R) = c_k(R_0) exp(-2 pi i (a i + b j) / M):
 *        Psi for all probes is one M x M DFT over the beam lattice per window pixel, and so is
 *        G Psi, from Z = G S_1w^T.  This replaces the products C S_1w (P_s K N_1) and G Psi
 *        (P_s K^2) by one K^2 N_1 product and FFTs; the same sums, regrouped exactly.  1
 *        (default) where it applies and needs fewer flops than the form chosen otherwise, 2
 *        wherever it applies, 0 never.
 * key 8: S_1 checkpoints between slice groups.  When the S_1 windows of all ionised slices
 *        do not fit the workspace budget, the slices form groups, and without checkpoints the
 *        forward sweep reruns from slice 0 for each group.  With them the first group's sweep
 *        saves the S_1 state at the entrance of every later group's lowest slice (N_1 x n_y x
 *        live columns complex64 per saved state, taken from the windows' share of the budget),
 *        and each later group resumes there.  The map is the same bit for bit.  1 (default)
 *        where the sweeps then cost fewer passes, 2 whenever there are several groups, 0 never.
 * key 9: the window-Gram form in split precision forms G = M o sum_t conj(H_t) H_t^T in the
 *        epilogue of the Gram GEMM (both triangles, in the SC format of the next product)
 *        instead of writing M and combining it in a separate pass: 1 (default) where every
 *        site has at most 32 transitions, 0 never.
 * key 10: tiles of that Gram GEMM with the G epilogue: 0 (default) 128 x 128 tiles of 4
 *        waves, 1 256 x 128 tiles of 8 waves.  Tiles with no element on or above the diagonal
 *        are skipped either way, and the maps are the same.
 * key 11: operand staging of the two-stage split GEMMs (16-complex tiles): 0 global_load_lds
 *        straight into the LDS ring everywhere; 1 (default) on the 256-row tiles, global loads
 *        into registers one tile ahead, written to the ring at the top of the next step (the
 *        nanoparticle map's Z product 2.86 -> 2.66 s); 2 that on the 128-row tiles too (its
 *        Gram tiles measured 2% slower so).  The maps are the same bit for bit.
 * Returns EELS_ERR_INVALID_ARG for an unknown key or an out-of-range value. */
eels_status eels_tune_set(int key, int value);
int eels_tune_get(int key);

/* Phase timing (diagnostics).  While enabled, eels_execute records HIP events on its
 * stream around each group of launches (at most `capacity` groups per call; further
 * groups are not timed).  After the stream has finished, eels_timing_read returns, for
 * the most recent eels_execute, the summed milliseconds and number of timed groups per
 * phase.  capacity 0 disables timing and releases the events.  Not thread-safe. */
enum {
    EELS_PHASE_SETUP = 0,     /* twiddles, T, P, probe coefficients                        */
    EELS_PHASE_SWEEP = 1,     /* row and column passes of both sweeps (with captures)      */
    EELS_PHASE_PRODUCER = 2,  /* band FFT / H-multiply producers                           */
    EELS_PHASE_GEMM1 = 3,     /* first contraction GEMM of each batch                      */
    EELS_PHASE_GEMM2 = 4,     /* second GEMM (detector |.|^2 epilogue; window Gram: G Psi)  */
    EELS_PHASE_REDUCE = 5,    /* FP64 per-probe reduction                                  */
    EELS_PHASE_IMAGES = 6,    /* elastic companion images (exit capture excluded)          */
    EELS_PHASE_GRAM = 7,      /* window-Gram form: Gram GEMM of each site's S_2 window     */
    EELS_PHASE_RASTER = 8,    /* raster form: the DFTs of Psi and Y over the beam lattice  */
    EELS_PHASES = 9
};
eels_status eels_timing_enable(int capacity);
eels_status eels_timing_read(double* ms, int* counts);

#ifdef __cplusplus
}
#endif
#endif /* EELS_H */
