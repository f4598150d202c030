// Host check of the planner (plan.cpp), built with AddressSanitizer and UndefinedBehaviorSanitizer
// by tests/test_plan_sanitized.py.  It plans a matrix of problems (grid sides 64 .. 512 and 384,
// crop windows and full cells, interpolation factors 1 .. 4, both contraction orders, the Gram,
// window-Gram and raster forms, every precision, slice groups under a memory budget, resident
// S-matrices, the inverse multislice, companion images, 256-row tiles) plus invalid problems, and
// checks each plan's tables against the buffers the device path addresses with them:
//   - workspace buffers in order, 256-byte aligned, inside workspace_bytes;
//   - every table offset inside the blob, the descriptor copy in the blob equal to descs;
//   - per batch: descriptor and job ranges, cumulative tile starts and tile totals;
//   - per launched descriptor: the rows and columns its kernel reads from A, B and H and writes to
//     C or the partial sums, through its gather index where it has one, inside the buffer that
//     launch binds (the same binding the contraction uses: by order, detector-sum form,
//     precision and which GEMM of the batch);
//   - the reduction CSR (monotone, entries inside the descriptors and partial sums);
//   - the capture CSRs of both sweeps (records inside the window buffers);
//   - the raster tables (beam permutation, slot positions, probe residues, DFT-block partials).
// Exit status 0 and "plan_check: N cases ok" when every check holds; otherwise each failure is
// printed and the status is 1.  No device code is involved.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace eels {
static std::string g_err_text;
static int g_knobs[TUNE_COUNT] = {0};
void set_error(const std::string& m) { g_err_text = m; }
int tune_get(int key) { return (key >= 0 && key < TUNE_COUNT) ? g_knobs[key] : 0; }
}  // namespace eels

using namespace eels;

namespace {

int g_failures = 0;
std::string g_case;
long g_descs = 0, g_batches = 0, g_entries = 0, g_plans = 0, g_raster = 0, g_wgram = 0, g_gram = 0, g_groups = 0,
     g_ckpt = 0;

#define CHECK(cond, ...)                                               \
    do {                                                               \
        if (!(cond)) {                                                 \
            ++g_failures;                                              \
            std::fprintf(stderr, "[%s] check failed: %s: ", g_case.c_str(), #cond); \
            std::fprintf(stderr, __VA_ARGS__);                         \
            std::fprintf(stderr, "\n");                                \
        }                                                              \
    } while (0)

struct Case {
    std::string name;
    int n = 128;
    double dx = 0.25;
    int nz = 6;
    int f = 1;
    double window_A = 0;
    int n_sites = 6, trans = 3;
    int px = 8, py = 8;
    double step = 0;           // probe step (A); 0: L / px
    int precision = EELS_FP32, order = EELS_ORDER_AUTO, detsum = EELS_DETSUM_AUTO;
    int s1_mode = EELS_S1_STORED, resident = 0, real_space = 0, n_images = 0;
    size_t budget = 0;
    bool tight_budget = false; // the budget is the smallest one the planner accepts (bisection)
    double budget_frac = 0;    // > 0: the budget is this fraction of the unconstrained workspace
    double aperture = 20, det_in = 10, det_out = 40;
    int knobs[TUNE_COUNT] = {0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 0, 1};
    eels_status expect = EELS_OK;
    int want_raster = -1, want_wgram = -1, want_gram = -1, want_groups_gt1 = -1, want_ckpt = -1;
};

enum Buf { B_NONE, B_W1, B_W2, B_C, B_MID, B_MID2, B_PART, B_IMG_MASKED, B_IMG_PART, B_H, B_COUNT };
const char* buf_name[B_COUNT] = {"-", "w1", "w2", "C", "mid", "mid2", "part", "img_masked", "img_part", "H"};

struct Sizes {
    int64_t e[B_COUNT] = {0};   // elements of 8 bytes (part: floats)
};

// One GEMM launch binding: source buffers of A, B (and H), destination of C or the partials,
// the kernel family (split SC or FP32 with B as rows (kind 0) or as [k][n] (kind 1)) and epilogue.
struct Role {
    Buf a = B_NONE, b = B_NONE, h = B_NONE, c = B_NONE, p = B_NONE;
    bool split = false;
    int kind = 0;
    int epi = 0;   // 0/3 store C, 1 norm partials (floats), 2 Gram tiles (float2 into p), 4 G (SC into c)
};

int64_t blob_ints(const Plan& p) { return (int64_t)p.blob.size(); }

bool in_blob(const Plan& p, int64_t off, int64_t n) { return off >= 0 && n >= 0 && off + n <= blob_ints(p); }

const int32_t* blob_at(const Plan& p, int64_t off) { return p.blob.data() + off; }

// rows of the gathered operand: index values (from the blob) or 0 .. n-1
int64_t max_row(const Plan& p, int64_t idx_off, int n, const char* what) {
    if (n <= 0) return -1;
    if (idx_off < 0) return n - 1;
    if (!in_blob(p, idx_off, n)) {
        CHECK(false, "%s gather index [%lld, +%d) outside the blob (%lld ints)", what, (long long)idx_off, n,
              (long long)blob_ints(p));
        return -1;
    }
    int64_t m = -1;
    const int32_t* ix = blob_at(p, idx_off);
    for (int i = 0; i < n; ++i) {
        CHECK(ix[i] >= 0, "%s gather index %d negative", what, i);
        m = std::max<int64_t>(m, ix[i]);
    }
    return m;
}

void check_extent(const char* what, int di, Buf b, int64_t end, const Sizes& sz) {
    CHECK(b != B_NONE, "descriptor %d: %s has no buffer", di, what);
    if (b == B_NONE) return;
    CHECK(end <= sz.e[b], "descriptor %d: %s reaches element %lld of %s (%lld elements)", di, what, (long long)end,
          buf_name[b], (long long)sz.e[b]);
}

void check_desc(const Plan& p, int di, const Role& r, const Sizes& sz) {
    const GemmDesc& d = p.descs[di];
    ++g_descs;
    CHECK(d.M > 0 && d.N_inner > 0 && d.K > 0 && d.n_t > 0, "descriptor %d: empty problem launched", di);
    if (!(d.M > 0 && d.N_inner > 0 && d.K > 0 && d.n_t > 0)) return;
    CHECK(d.tiles_n == (int)ceil_div(d.N_inner, GEMM_BN), "descriptor %d: tiles_n", di);
    CHECK(d.a_off >= 0 && d.b_off >= 0, "descriptor %d: negative operand offset", di);
    const int64_t t1 = d.n_t - 1;
    const bool idx_a = r.split ? (d.flags & GD_IDX_A) != 0 : (r.kind == 1 && d.idx_off >= 0);
    const bool idx_b = d.idx_off >= 0 && !idx_a;
    const int64_t kr = r.split ? round_up(d.K, 16) : round_up(d.K, 2);   // columns the loads touch
    const int64_t am = max_row(p, idx_a ? d.idx_off : -1, d.M, "A");
    check_extent("A", di, r.a, d.a_off + t1 * d.a_tstride + am * d.lda + kr, sz);
    if (!r.split && r.kind == 1) {
        check_extent("B ([k][n])", di, r.b, d.b_off + t1 * d.b_tstride + (int64_t)(d.K - 1) * d.ldb + round_up(d.N_inner, 2), sz);
        CHECK(!idx_b, "descriptor %d: kind-1 B cannot be gathered", di);
    } else {
        const int64_t bm = max_row(p, idx_b ? d.idx_off : -1, d.N_inner, "B");
        check_extent("B", di, r.b, d.b_off + t1 * d.b_tstride + bm * d.ldb + kr, sz);
    }
    if (d.h_off >= 0 && !r.split && r.h != B_NONE) check_extent("H", di, r.h, d.h_off + t1 * d.ldh + d.K, sz);
    if (d.lda < d.K || (r.kind == 0 && d.ldb < d.K)) CHECK(false, "descriptor %d: leading dimension below K", di);
    if (r.epi == 0 || r.epi == 3) {
        const bool pad = r.split || (d.flags & GD_ZERO_PAD);
        const int64_t ncols = pad ? round_up(d.N_inner, 16) : d.N_inner;
        check_extent("C", di, r.c, d.c_off + t1 * d.ldc_t + (int64_t)(d.M - 1) * d.ldc_m + ncols, sz);
        CHECK(d.ldc_m >= ncols || d.M == 1, "descriptor %d: C rows overlap (ldc_m %lld < %lld)", di,
              (long long)d.ldc_m, (long long)ncols);
    } else if (r.epi == 1) {
        check_extent("partials", di, r.p, d.p_off + (int64_t)(d.tiles_m - 1) * d.ld_part + t1 * d.N_inner + d.N_inner, sz);
        CHECK(d.ld_part >= (int64_t)d.n_t * d.N_inner, "descriptor %d: partial rows overlap", di);
    } else if (r.epi == 2) {
        // float2 Gram tiles: for the part buffer (floats) count in floats
        const int64_t end = d.p_off + t1 * d.ldc_t + (int64_t)(d.M - 1) * d.ldc_m + d.N_inner;
        check_extent("Gram tiles", di, r.p, r.p == B_PART ? 2 * end : end, sz);
    } else if (r.epi == 4) {
        // G in SC, both triangles of the square: every row N .. ldc_m - 1 padded; H of ld_part
        // transitions, ldh apart
        CHECK(d.M == d.N_inner && d.ldc_m >= round_up(d.N_inner, 16) && d.ldc_m % 4 == 0,
              "descriptor %d: G tile shape", di);
        check_extent("G", di, r.c, d.c_off + (int64_t)(d.M - 1) * d.ldc_m + d.ldc_m, sz);
        CHECK(d.ld_part >= 1 && d.ld_part <= 32 && d.ldh >= d.M, "descriptor %d: %lld transitions", di,
              (long long)d.ld_part);
        check_extent("H", di, r.h, d.h_off + (d.ld_part - 1) * d.ldh + d.M, sz);
    }
}

// the launch bindings of the contraction (which buffers each GEMM of a batch reads and writes)
Role role_d1(const Plan& p) {
    const bool split = p.precision != EELS_FP32, orderS = p.order == EELS_ORDER_S_FIRST, h_pro = !p.recip;
    Role r;
    r.split = split;
    r.c = B_MID;
    if (p.gram) { r.a = B_MID2; r.b = B_W2; r.epi = 0; }
    else if (orderS) {
        r.a = B_W2; r.b = split ? B_MID2 : (h_pro ? B_W1 : B_MID2); r.h = (!split && h_pro) ? B_H : B_NONE; r.epi = 0;
    } else {
        r.a = B_C;
        if (split) { r.b = B_MID2; r.epi = p.hs2 ? 0 : 3; }
        else { r.b = B_W1; r.kind = 1; r.epi = 0; }
    }
    return r;
}

Role role_d2(const Plan& p) {
    const bool split = p.precision != EELS_FP32, orderS = p.order == EELS_ORDER_S_FIRST, h_pro = !p.recip;
    Role r;
    r.split = split;
    r.p = B_PART;
    if (p.gram) { r.a = B_MID; r.b = B_MID; r.epi = 2; }
    else if (orderS) { r.a = B_MID; r.b = B_C; r.epi = 1; }
    else if (split && p.hs2) { r.a = B_MID2; r.b = B_MID; r.epi = 1; }
    else if (split) { r.a = B_W2; r.b = B_MID2; r.epi = 1; }
    else { r.a = B_W2; r.b = h_pro ? B_MID : B_MID2; r.h = h_pro ? B_H : B_NONE; r.epi = 1; }
    return r;
}

Role role_dm(const Plan& p) {
    Role r;
    r.split = p.precision != EELS_FP32;
    r.a = r.b = r.p = B_MID2;
    r.epi = 2;
    if (p.wg_fused) { r.epi = 4; r.c = B_MID2; r.h = B_H; }
    return r;
}

Role role_dy(const Plan& p) {
    Role r;
    r.split = p.precision != EELS_FP32;
    r.c = B_MID2;
    r.epi = r.split ? 3 : 0;
    if (p.raster) { r.a = B_MID2; r.b = (r.split && !p.w1_sc) ? B_MID2 : B_W1; }
    else { r.a = B_MID; r.b = B_MID2; }
    return r;
}

void check_reduction_entry(const Plan& p, const Batch& b, int desc, int col, const Sizes& sz) {
    const bool in_range = desc >= b.d2_begin && desc < b.d2_begin + b.d2_count;
    CHECK(in_range, "reduction entry names descriptor %d outside the batch's second GEMM", desc);
    if (!in_range) return;
    const GemmDesc& d = p.descs[desc];
    CHECK(col >= 0 && col < d.N_inner, "reduction column %d outside N_inner %d", col, d.N_inner);
    const int64_t end = d.p_off + (int64_t)(d.tiles_m - 1) * d.ld_part + (int64_t)(d.n_t - 1) * d.N_inner + col + 1;
    CHECK(end <= sz.e[B_PART], "reduction reads partial %lld of %lld", (long long)end, (long long)sz.e[B_PART]);
}

void check_capture(const Plan& p, int j, int64_t ptr_off, int64_t rec_off, int which) {
    CHECK(in_blob(p, ptr_off, p.ny + 1), "slice %d capture %d row pointers outside the blob", j, which);
    if (!in_blob(p, ptr_off, p.ny + 1)) return;
    const int32_t* ptr = blob_at(p, ptr_off);
    CHECK(ptr[0] == 0, "slice %d capture %d starts at %d", j, which, ptr[0]);
    for (int y = 0; y < p.ny; ++y) CHECK(ptr[y + 1] >= ptr[y], "slice %d capture %d not monotone at row %d", j, which, y);
    const int n = ptr[p.ny];
    CHECK(in_blob(p, rec_off, 4 * (int64_t)n), "slice %d capture %d records outside the blob", j, which);
    if (!in_blob(p, rec_off, 4 * (int64_t)n)) return;
    const int32_t* rec = blob_at(p, rec_off);
    const int64_t beams = which == 0 ? p.N1 : p.N2;
    const int64_t win_cap = which == 0 ? std::max(p.max_w1, 1)
                                       : (p.resident ? (int64_t)std::max(p.max_w2, 1)
                                                     : (int64_t)std::max(p.max_w2, 1));
    for (int i = 0; i < n; ++i) {
        const int win = rec[4 * i], dy = rec[4 * i + 1], x0 = rec[4 * i + 2], nwx = rec[4 * i + 3];
        CHECK(win >= 0 && win < win_cap, "slice %d capture %d record %d: window %d of %lld", j, which, i, win,
              (long long)win_cap);
        CHECK(dy >= 0 && x0 >= 0 && x0 < p.nx && nwx >= 1 && nwx <= p.nx, "slice %d capture %d record %d fields", j,
              which, i);
        CHECK((int64_t)(dy + 1) * nwx <= p.K && p.K <= p.Kpad, "slice %d capture %d record %d: window row %d leaves K",
              j, which, i, dy);
    }
    (void)beams;
}

void check_plan(const Plan& p, const Case& c, size_t budget) {
    // ---- workspace layout
    const size_t offs[] = {p.off_twx, p.off_twy, p.off_T, p.off_P, p.off_s1, p.off_s2, p.off_w1, p.off_w2, p.off_C,
                           p.off_mid, p.off_mid2, p.off_scratch, p.off_part, p.off_gtot, p.off_qpart,
                           p.off_img_exit, p.off_img_masked, p.off_img_part, p.off_img_G, p.off_img_qpart,
                           p.off_img_C, p.off_r_c0, p.off_r_tw, p.off_ckpt, p.off_blob};
    const int n_offs = (int)(sizeof(offs) / sizeof(offs[0]));
    for (int i = 0; i < n_offs; ++i) {
        CHECK(offs[i] % 256 == 0, "workspace buffer %d at %zu not 256-byte aligned", i, offs[i]);
        if (i > 0) CHECK(offs[i] >= offs[i - 1], "workspace buffer %d before buffer %d", i, i - 1);
    }
    CHECK(p.off_blob + 4 * p.blob.size() <= p.ws_bytes, "blob beyond workspace_bytes");
    if (budget > 0) CHECK(p.ws_bytes <= budget, "workspace %zu over the budget %zu", p.ws_bytes, budget);
    CHECK(p.off_s1 + 8 * (size_t)p.N1 * p.ny * p.ldx <= p.off_s2, "S_1 state overlaps S_2");
    CHECK(p.ldx >= p.nlx && p.ldx % 16 == 0, "ldx %d for %d live columns", p.ldx, p.nlx);
    // S_1 checkpoints: one slot per later group that resumes above slice 0, saved at that
    // slice's entrance by the first group's sweep (which must pass it), all inside their region
    {
        const size_t slot = (8 * (size_t)p.N1 * p.ny * p.ldx + 255) / 256 * 256;
        CHECK(p.n_ckpt == 0 || p.off_ckpt + (size_t)p.n_ckpt * slot <= p.off_blob, "checkpoints overlap the blob");
        int seen = 0;
        for (size_t g = 0; g < p.groups.size(); ++g) {
            const Group& gr = p.groups[g];
            CHECK(gr.j_lo <= gr.j_hi, "group %zu slices %d..%d", g, gr.j_lo, gr.j_hi);
            if (g > 0) CHECK(gr.j_hi < p.groups[g - 1].j_lo, "group %zu not below group %zu", g, g - 1);
            if (gr.ckpt < 0) continue;
            ++seen;
            CHECK(g > 0 && gr.j_lo > 0 && gr.ckpt < p.n_ckpt, "group %zu checkpoint %d", g, gr.ckpt);
            CHECK(gr.j_lo <= p.groups[0].j_hi, "checkpoint of group %zu above the first group's sweep", g);
            CHECK(p.slices[gr.j_lo].ckpt_save == gr.ckpt, "slice %d saves slot %d, group %zu reads %d", gr.j_lo,
                  p.slices[gr.j_lo].ckpt_save, g, gr.ckpt);
        }
        CHECK(seen == p.n_ckpt, "%d groups read checkpoints, %d slots", seen, p.n_ckpt);
        if (p.resident) CHECK(p.n_ckpt == 0, "resident plan with checkpoints");
    }

    Sizes sz;
    sz.e[B_W1] = (int64_t)std::max(p.max_w1, 1) * p.N1 * p.Kpad;
    sz.e[B_W2] = (int64_t)(p.off_C - p.off_w2) / 8;
    sz.e[B_C] = (int64_t)p.P * p.N1pad;
    sz.e[B_MID] = std::max<int64_t>(p.mid_elems, 1);
    sz.e[B_MID2] = std::max<int64_t>(p.mid2_elems, 1);
    sz.e[B_PART] = std::max<int64_t>(p.part_elems, 1);
    sz.e[B_IMG_MASKED] = p.n_img > 0 ? (int64_t)p.N1 * p.Kbpad : 0;
    sz.e[B_IMG_PART] = p.n_img > 0 ? (int64_t)p.N1pad * p.N1pad : 0;
    sz.e[B_H] = p.n_trans_total * (int64_t)p.K;
    CHECK((int64_t)(p.off_w1 + 8 * (size_t)sz.e[B_W1]) <= (int64_t)p.off_w2, "w1 overlaps w2");
    CHECK((int64_t)(p.off_mid + 8 * (size_t)sz.e[B_MID]) <= (int64_t)p.off_mid2, "mid overlaps mid2");
    CHECK((int64_t)(p.off_mid2 + 8 * (size_t)sz.e[B_MID2]) <= (int64_t)p.off_scratch, "mid2 overlaps scratch");
    CHECK((int64_t)(p.off_part + 4 * (size_t)sz.e[B_PART]) <= (int64_t)p.off_gtot, "part overlaps gtot");

    // ---- table offsets inside the blob
    const int64_t tables[][2] = {{p.b1_off, 4 * (int64_t)p.N1}, {p.b2_off, 4 * (int64_t)p.N2}, {p.ident_off, p.P},
                                 {p.band_h_off, p.nlx}, {p.band_off_off, p.nlx}, {p.dz_off, 2 * (int64_t)p.nz},
                                 {p.probes_off, 4 * (int64_t)p.P}, {p.dbg_ptr, p.ny + 1}, {p.dbg_rec, 4 * (int64_t)p.ny},
                                 {p.det_mask_off, p.Kbpad}, {p.col_ptr_off, p.nlx + 1}, {p.col_beam_off, 1},
                                 {p.conv_org_off, 4}};
    for (const auto& t : tables) CHECK(in_blob(p, t[0], t[1]), "table at %lld (+%lld) outside the blob", (long long)t[0], (long long)t[1]);
    CHECK(in_blob(p, p.descs_off, (int64_t)p.descs.size() * (int64_t)(sizeof(GemmDesc) / 4)), "descriptor table outside the blob");
    if (in_blob(p, p.descs_off, (int64_t)p.descs.size() * (int64_t)(sizeof(GemmDesc) / 4)) && !p.descs.empty())
        CHECK(std::memcmp(blob_at(p, p.descs_off), p.descs.data(), p.descs.size() * sizeof(GemmDesc)) == 0,
              "descriptor copy in the blob differs");
    CHECK(p.descs_off % 4 == 0 && p.dz_off % 2 == 0 && p.probes_off % 2 == 0, "16-byte table alignment");
    // beams of the sweeps: live column and row inside the grid
    if (in_blob(p, p.b1_off, 4 * (int64_t)p.N1))
        for (int b = 0; b < p.N1; ++b) {
            const int32_t* e = blob_at(p, p.b1_off + 4 * (int64_t)b);
            CHECK(e[0] >= 0 && e[0] < p.nlx && e[1] >= 0 && e[1] < p.ny, "aperture beam %d at (%d, %d)", b, e[0], e[1]);
        }
    if (in_blob(p, p.b2_off, 4 * (int64_t)p.N2))
        for (int b = 0; b < p.N2; ++b) {
            const int32_t* e = blob_at(p, p.b2_off + 4 * (int64_t)b);
            CHECK(e[0] >= 0 && e[0] < p.nlx && e[1] >= 0 && e[1] < p.ny, "detector beam %d at (%d, %d)", b, e[0], e[1]);
        }
    if (in_blob(p, p.col_ptr_off, p.nlx + 1)) {
        const int32_t* cp = blob_at(p, p.col_ptr_off);
        CHECK(cp[0] == 0 && cp[p.nlx] == p.N1, "aperture beams by column: %d .. %d of %d", cp[0], cp[p.nlx], p.N1);
    }
    int64_t band_end = 0;
    for (int cidx = 0; cidx < p.nlx; ++cidx) band_end = std::max<int64_t>(band_end, p.band_off[cidx] + 2 * p.band_h[cidx] + 1);
    CHECK(band_end <= p.Kbpad, "band slots %lld beyond Kbpad %d", (long long)band_end, p.Kbpad);

    // ---- capture CSRs of the ionised slices
    for (int j = 0; j < p.nz; ++j) {
        const SliceInfo& si = p.slices[j];
        if (!si.ion) continue;
        check_capture(p, j, si.cap1_ptr, si.cap1_rec, 0);
        if (!p.recip) check_capture(p, j, si.cap2_ptr, si.cap2_rec, 1);
        const int64_t w2_slice = p.recip ? (int64_t)p.N2 * p.Kbpad : (int64_t)std::max(p.max_w2, 1) * p.N2 * p.Kpad;
        CHECK(p.slice_w2[j] + w2_slice <= sz.e[B_W2], "slice %d S_2 capture leaves w2", j);
    }
    for (size_t s = 0; s < p.sites.size(); ++s) {
        if (p.site_w1[s] < 0 && p.site_w2[s] < 0) continue;   // skipped: no transitions or no eligible probe
        CHECK(p.site_w1[s] >= 0 && p.site_w1[s] < std::max(p.max_w1, 1), "site %zu S_1 window %d", s, p.site_w1[s]);
        CHECK(p.site_w2[s] >= 0 && p.site_w2[s] < std::max(p.max_w2, 1), "site %zu S_2 window %d", s, p.site_w2[s]);
    }

    // ---- batches
    const Role r1 = role_d1(p), r2 = role_d2(p), rm = role_dm(p), ry = role_dy(p);
    const int nd = (int)p.descs.size();
    ++g_plans;
    g_raster += p.raster; g_wgram += p.wgram; g_gram += p.gram; g_groups += p.groups.size() > 1;
    g_ckpt += p.n_ckpt > 0;
    for (size_t bi = 0; bi < p.batches.size(); ++bi) {
        const Batch& b = p.batches[bi];
        ++g_batches;
        struct Range { int begin, count, tiles; const Role* role; const char* name; bool launched; };
        const Range ranges[] = {{b.d1_begin, b.d1_count, b.d1_tiles, &r1, "first GEMM", true},
                                {b.d2_begin, b.d2_count, b.d2_tiles, &r2, "second GEMM", !p.wgram},
                                {b.dm_begin, b.dm_count, b.dm_tiles, &rm, "window Gram", p.wgram},
                                {b.dy_begin, b.dy_count, b.dy_tiles, &ry, "G product", p.wgram}};
        for (const Range& rg : ranges) {
            CHECK(rg.begin >= 0 && rg.count >= 0 && rg.begin + rg.count <= nd, "batch %zu %s range", bi, rg.name);
            if (!(rg.begin >= 0 && rg.count >= 0 && rg.begin + rg.count <= nd)) continue;
            int tiles = 0;
            for (int k = 0; k < rg.count; ++k) {
                const GemmDesc& d = p.descs[rg.begin + k];
                CHECK(d.tile_start == tiles, "batch %zu %s descriptor %d tile_start %d, expected %d", bi, rg.name, k,
                      d.tile_start, tiles);
                tiles += d.tiles_m * d.tiles_n * d.n_t;
                if (rg.launched) check_desc(p, rg.begin + k, *rg.role, sz);
            }
            CHECK(tiles == rg.tiles, "batch %zu %s: %d tiles, table says %d", bi, rg.name, tiles, rg.tiles);
            // row tiles of the launch (128 or 256 rows)
            const int rows = rg.role == &r1 ? b.d1_rows : rg.role == &r2 ? b.d2_rows : rg.role == &ry ? b.dy_rows : b.dm_rows;
            CHECK(rows == 128 || rows == 256, "batch %zu %s rows %d", bi, rg.name, rows);
            for (int k = 0; k < rg.count && rg.launched; ++k) {
                const GemmDesc& d = p.descs[rg.begin + k];
                CHECK(d.tiles_m == (int)ceil_div(d.M, rows), "batch %zu %s descriptor %d: %d row tiles of %d for M %d",
                      bi, rg.name, k, d.tiles_m, rows, d.M);
            }
        }
        CHECK(b.job_begin >= 0 && b.job_begin + b.job_count <= (int)p.jobs.size(), "batch %zu job range", bi);
        for (int k = 0; k < b.job_count; ++k) {
            const Job& jb = p.jobs[b.job_begin + k];
            // the window-Gram producers read the S_2 window (the ProdJob's s2w)
            const Buf src = (p.wgram || jb.from_mid == 2) ? B_W2 : jb.from_mid ? B_MID : B_W1;
            CHECK(jb.w_off >= 0 && jb.w_off < sz.e[src], "batch %zu job %d source offset", bi, k);
            CHECK(jb.win_off >= 0 && jb.win_off < sz.e[B_W1], "batch %zu job %d window offset", bi, k);
            CHECK(jb.dst_off >= 0 && jb.dst_off < sz.e[B_MID2], "batch %zu job %d destination", bi, k);
            CHECK(jb.h_off >= 0 && jb.h_off + (int64_t)jb.nt * p.K <= sz.e[B_H], "batch %zu job %d transitions", bi, k);
        }
        // window-Gram and raster forms: every site's operands in mid2 (S_2w^T, the Gram tiles M, G,
        // Y or Z, and in the raster form Xt and the SC copy of S_1w) are disjoint, within the site
        // and across the batch's sites
        if (p.wgram) {
            struct Reg { int64_t a, e; const char* what; int job; };
            std::vector<Reg> regs;
            for (int k = 0; k < b.job_count; ++k) {
                const Job& jb = p.jobs[b.job_begin + k];
                regs.push_back({jb.s2t_off, jb.s2t_off + (int64_t)p.K * p.N2p, "S_2w^T", k});
                regs.push_back({jb.m_off, jb.m_off + (int64_t)p.K * p.Kpad, "M", k});
                regs.push_back({jb.g_off, jb.g_off + (int64_t)p.K * p.Kpad, "G", k});
                if (p.raster) {
                    regs.push_back({jb.y_off, jb.y_off + (int64_t)p.K * p.N1pad, "Z", k});
                    regs.push_back({jb.xt_off, jb.xt_off + (int64_t)p.K * p.N1pad, "Xt", k});
                    if (p.precision != EELS_FP32 && !p.w1_sc)
                        regs.push_back({jb.s1sc_off, jb.s1sc_off + (int64_t)p.N1 * p.Kpad, "S_1w SC", k});
                } else {
                    regs.push_back({jb.y_off, jb.y_off + (int64_t)std::max(jb.ps, 1) * p.Kpad, "Y^T", k});
                }
            }
            for (size_t u = 0; u < regs.size(); ++u)
                for (size_t v = u + 1; v < regs.size(); ++v)
                    CHECK(regs[u].e <= regs[v].a || regs[v].e <= regs[u].a,
                          "batch %zu: %s of site %d [%lld, %lld) overlaps %s of site %d [%lld, %lld)", bi, regs[u].what,
                          regs[u].job, (long long)regs[u].a, (long long)regs[u].e, regs[v].what, regs[v].job,
                          (long long)regs[v].a, (long long)regs[v].e);
        }
        // producer tables of the window-Gram and raster forms
        if (p.wgram) {
            const int64_t n = (int64_t)b.job_count * (int64_t)(sizeof(ProdJob) / 4);
            CHECK(in_blob(p, b.p_jobs, n) && b.p_jobs % 2 == 0, "batch %zu ProdJob table", bi);
            if (in_blob(p, b.p_jobs, n))
                for (int k = 0; k < b.job_count; ++k) {
                    ProdJob q;
                    std::memcpy(&q, blob_at(p, b.p_jobs) + k * (sizeof(ProdJob) / 4), sizeof(q));
                    const Job& jb = p.jobs[b.job_begin + k];
                    CHECK(q.s2w + (int64_t)(p.N2 - 1) * p.Kpad + p.K <= sz.e[B_W2], "batch %zu ProdJob %d S_2 window", bi, k);
                    CHECK(q.s1w + (int64_t)(p.N1 - 1) * p.Kpad + p.K <= sz.e[B_W1], "batch %zu ProdJob %d S_1 window", bi, k);
                    CHECK(q.s2t == jb.s2t_off && q.g == jb.g_off && q.m == jb.m_off && q.nt == jb.nt,
                          "batch %zu ProdJob %d differs from its job", bi, k);
                    CHECK(q.g + (int64_t)(p.K - 1) * p.Kpad + round_up(p.K, 16) <= sz.e[B_MID2], "batch %zu ProdJob %d G", bi, k);
                    CHECK(q.h + (int64_t)q.nt * p.K <= sz.e[B_H], "batch %zu ProdJob %d H", bi, k);
                }
        }
        if (p.raster) {
            const int64_t n = 6 * (int64_t)b.job_count;
            CHECK(in_blob(p, b.r_jobs, n) && b.r_jobs % 2 == 0, "batch %zu RasterJob table", bi);
            if (in_blob(p, b.r_jobs, n))
                for (int k = 0; k < b.job_count; ++k) {
                    RasterJob q;
                    std::memcpy(&q, blob_at(p, b.r_jobs) + 6 * k, sizeof(q));
                    const int64_t last = (int64_t)(p.K - 1) * p.N1pad + p.N1pad;
                    CHECK(q.xt >= 0 && q.xt + last <= sz.e[B_MID2], "batch %zu RasterJob %d Xt", bi, k);
                    CHECK(q.z >= 0 && q.z + last <= sz.e[B_MID2], "batch %zu RasterJob %d Z", bi, k);
                    CHECK(q.part >= 0 && q.part + (int64_t)p.r_chunks * p.rM * p.rM <= sz.e[B_PART],
                          "batch %zu RasterJob %d partials", bi, k);
                }
        }
        // reduction
        if (b.red_ptr >= 0) {
            CHECK(in_blob(p, b.red_ptr, p.P + 1), "batch %zu reduction pointers", bi);
            if (!in_blob(p, b.red_ptr, p.P + 1)) continue;
            const int32_t* rp = blob_at(p, b.red_ptr);
            CHECK(rp[0] == 0 && rp[p.P] == b.n_entries, "batch %zu reduction spans %d .. %d, %lld entries", bi, rp[0],
                  rp[p.P], (long long)b.n_entries);
            for (int r = 0; r < p.P; ++r) CHECK(rp[r + 1] >= rp[r], "batch %zu reduction not monotone at %d", bi, r);
            CHECK(in_blob(p, b.red_ent, 2 * b.n_entries), "batch %zu reduction entries", bi);
            if (!in_blob(p, b.red_ent, 2 * b.n_entries)) continue;
            const int32_t* en = blob_at(p, b.red_ent);
            for (int64_t e = 0; e < b.n_entries; ++e) check_reduction_entry(p, b, en[2 * e], en[2 * e + 1], sz);
            // raster form: every entry of probe r reads its residue's partial sums
            if (p.raster && (int)p.r_res.size() == p.P)
                for (int r = 0; r < p.P; ++r)
                    for (int e = rp[r]; e < rp[r + 1]; ++e)
                        CHECK(en[2 * e + 1] == p.r_res[r], "batch %zu probe %d reads residue %d, not %d", bi, r,
                              en[2 * e + 1], p.r_res[r]);
            g_entries += b.n_entries;
        } else if (!p.gram) {
            for (int k = 0; k < b.d2_count; ++k) {
                const GemmDesc& d = p.descs[b.d2_begin + k];
                CHECK(d.N_inner == p.P, "batch %zu dense reduction over %d columns for %d probes", bi, d.N_inner, p.P);
                check_reduction_entry(p, b, b.d2_begin + k, p.P - 1, sz);
            }
        } else {
            CHECK(2 * (int64_t)b.n_parts * p.N1pad * p.N1pad <= sz.e[B_PART], "batch %zu Gram partials", bi);
        }
    }
    if (p.n_img > 0) {
        CHECK(p.img_desc >= 0 && p.img_desc < nd, "image descriptor");
        if (p.img_desc >= 0 && p.img_desc < nd) {
            Role ri;
            ri.a = ri.b = B_IMG_MASKED; ri.p = B_IMG_PART; ri.epi = 2;
            check_desc(p, p.img_desc, ri, sz);
        }
        CHECK(in_blob(p, p.img_mask_off, p.Kbpad), "image ring masks");
    }

    // ---- raster tables
    if (p.raster) {
        const int M = p.rM;
        CHECK(M == 64 && p.r_chunk > 0 && p.r_chunks == (int)ceil_div(p.K, p.r_chunk), "raster sizes");
        CHECK((int)p.r_res.size() == p.P, "raster residues per probe");
        for (int r = 0; r < (int)p.r_res.size(); ++r) CHECK(p.r_res[r] >= 0 && p.r_res[r] < M * M, "probe %d residue %d", r, p.r_res[r]);
        CHECK(in_blob(p, p.r_perm_off, p.N1) && in_blob(p, p.r_pos_off, (int64_t)M * M), "raster tables in the blob");
        if (in_blob(p, p.r_perm_off, p.N1) && in_blob(p, p.r_pos_off, (int64_t)M * M)) {
            const int32_t* perm = blob_at(p, p.r_perm_off);
            const int32_t* pos = blob_at(p, p.r_pos_off);
            std::vector<int> seen(p.N1, 0);
            for (int q = 0; q < p.N1; ++q) {
                CHECK(perm[q] >= 0 && perm[q] < p.N1, "slot column %d holds beam %d", q, perm[q]);
                if (perm[q] >= 0 && perm[q] < p.N1) ++seen[perm[q]];
            }
            for (int b = 0; b < p.N1; ++b) CHECK(seen[b] == 1, "beam %d in %d slot columns", b, seen[b]);
            int filled = 0;
            for (int s = 0; s < M * M; ++s) {
                const int q = pos[s];
                CHECK(q >= -1 && q < p.N1, "grid slot %d at column %d", s, q);
                if (q < 0 || q >= p.N1) continue;
                ++filled;
                const int beam = perm[q];
                if (beam < 0 || beam >= p.N1) continue;
                const int a = p.ab1[2 * beam], bb = p.ab1[2 * beam + 1];
                const int slot = (((bb % M) + M) % M) * M + (((a % M) + M) % M);
                CHECK(slot == s, "grid slot %d holds beam (%d, %d) of slot %d", s, a, bb, slot);
            }
            CHECK(filled == p.N1, "%d grid slots for %d beams", filled, p.N1);
        }
        CHECK(p.off_r_tw >= p.off_r_c0 + 8 * (size_t)p.N1pad && p.off_blob >= p.off_r_tw + 8 * (size_t)M,
              "raster twiddles and probe phases");
    }

    // ---- expectations of the case
    if (c.want_raster >= 0) CHECK((int)p.raster == c.want_raster, "raster form %d, expected %d", (int)p.raster, c.want_raster);
    // SC S_1 windows exactly for the raster form in split precision without resident S-matrices
    CHECK(p.w1_sc == ((p.raster && p.precision != EELS_FP32 && !p.resident) ? p.precision : 0),
          "S_1 window format %d", p.w1_sc);
    if (c.want_wgram >= 0) CHECK((int)p.wgram == c.want_wgram, "window-Gram form %d, expected %d", (int)p.wgram, c.want_wgram);
    if (c.want_gram >= 0) CHECK((int)p.gram == c.want_gram, "Gram form %d, expected %d", (int)p.gram, c.want_gram);
    if (c.want_groups_gt1 >= 0)
        CHECK(((int)p.groups.size() > 1) == (c.want_groups_gt1 != 0), "%zu slice groups", p.groups.size());
    if (c.want_ckpt >= 0) CHECK((p.n_ckpt > 0) == (c.want_ckpt != 0), "%d checkpoints", p.n_ckpt);
    (void)s_signature(p);
}

uint32_t lcg(uint32_t& s) { s = s * 1664525u + 1013904223u; return s >> 8; }

void run_case(const Case& c) {
    g_case = c.name;
    std::memcpy(g_knobs, c.knobs, sizeof(g_knobs));
    const double L = c.n * c.dx;
    std::vector<double> dz(std::max(c.nz, 1), 2.0);
    std::vector<double> probes;
    const double step = c.step > 0 ? c.step : L / c.px;
    for (int j = 0; j < c.py; ++j)
        for (int i = 0; i < c.px; ++i) {
            probes.push_back(0.3 * L + i * step);
            probes.push_back(0.3 * L + j * step);
        }
    std::vector<eels_site> sites;
    uint32_t seed = 12345u + (uint32_t)c.n * 7u + (uint32_t)c.n_sites;
    int64_t h = 0;
    for (int s = 0; s < c.n_sites; ++s) {
        eels_site st{};
        st.slice = (int)(lcg(seed) % (uint32_t)std::max(c.nz, 1));
        st.n_trans = s % 5 == 4 ? 0 : 1 + (int)(lcg(seed) % (uint32_t)c.trans);
        st.x_A = (lcg(seed) % 10000) * 1e-4 * L;
        st.y_A = (lcg(seed) % 10000) * 1e-4 * L;
        st.h_offset = h;
        h += st.n_trans;
        sites.push_back(st);
    }
    const double img[4] = {0.0, 10.0, 40.0, 0.0};
    eels_problem q{};
    q.nx = q.ny = c.n;
    q.lx_A = q.ly_A = L;
    q.n_slices = c.nz;
    q.dz_A = dz.data();
    q.energy_eV = 80e3;
    q.aperture_mrad = c.aperture;
    q.det_inner_mrad = c.det_in;
    q.det_outer_mrad = c.det_out;
    q.defocus_A = 0;
    q.cs_A = 0;
    q.interp_f = c.f;
    q.window_A = c.window_A;
    q.n_probes = c.px * c.py;
    q.probe_xy = probes.empty() ? nullptr : probes.data();
    q.n_sites = c.n_sites;
    q.sites = sites.empty() ? nullptr : sites.data();
    q.n_trans_total = h;
    q.precision = c.precision;
    q.order = c.order;
    q.max_workspace_bytes = c.budget;
    q.real_space = c.real_space;
    q.resident_s = c.resident;
    q.detector_sum = c.detsum;
    q.s1_mode = c.s1_mode;
    q.n_images = c.n_images;
    q.image_detectors_mrad = c.n_images > 0 ? img : nullptr;
    Plan p;
    if (c.tight_budget) {
        // every budget between the refusals and the unconstrained workspace: bisect to the
        // smallest accepted one (each refusal is an OOM status, not a fault)
        CHECK(build_plan(p, q) == EELS_OK, "unconstrained plan: %s", g_err_text.c_str());
        size_t lo = 0, hi = p.ws_bytes;
        while (hi - lo > (hi >> 12) + 1) {
            const size_t mid = lo + (hi - lo) / 2;
            q.max_workspace_bytes = mid;
            const eels_status st = build_plan(p, q);
            CHECK(st == EELS_OK || st == EELS_ERR_OOM, "budget %zu: status %d", mid, (int)st);
            if (st == EELS_OK) hi = mid;
            else lo = mid;
        }
        q.max_workspace_bytes = hi;
    } else if (c.budget_frac > 0) {
        CHECK(build_plan(p, q) == EELS_OK, "unconstrained plan: %s", g_err_text.c_str());
        q.max_workspace_bytes = (size_t)(c.budget_frac * (double)p.ws_bytes);
    }
    const eels_status s = build_plan(p, q);
    CHECK(s == c.expect, "status %d (%s), expected %d", (int)s, g_err_text.c_str(), (int)c.expect);
    if (s == EELS_OK) check_plan(p, c, q.max_workspace_bytes);
}

Case mk(const char* name) { Case c; c.name = name; return c; }

}  // namespace

int main() {
    std::vector<Case> cases;
    const int precs[] = {EELS_FP32, EELS_BF16_SPLIT, EELS_FP16_SPLIT};
    for (int prec : precs) {
        const std::string ps = prec == EELS_FP32 ? "fp32" : prec == EELS_BF16_SPLIT ? "bf16" : "fp16";
        // full cell, f = 1: band basis, order S or Gram form
        { Case c = mk(""); c.name = "full-" + ps; c.precision = prec; cases.push_back(c); }
        { Case c = mk(""); c.name = "full-gram-" + ps; c.precision = prec; c.detsum = EELS_DETSUM_GRAM;
          c.want_gram = 1; cases.push_back(c); }
        { Case c = mk(""); c.name = "full-direct-orderS-" + ps; c.precision = prec; c.detsum = EELS_DETSUM_DIRECT;
          c.order = EELS_ORDER_S_FIRST; c.want_gram = 0; cases.push_back(c); }
        { Case c = mk(""); c.name = "full-real-space-" + ps; c.precision = prec; c.real_space = 1; c.n = 64;
          c.order = EELS_ORDER_S_FIRST; cases.push_back(c); }
        // crop windows, f = 1 .. 4, both orders, window-Gram and direct
        for (int f : {1, 2, 4}) {
            for (int order : {EELS_ORDER_S_FIRST, EELS_ORDER_PROBE_FIRST}) {
                for (int wg : {0, 2}) {
                    Case c = mk("");
                    c.name = "crop-f" + std::to_string(f) + (order == EELS_ORDER_S_FIRST ? "-S" : "-P") +
                             (wg ? "-wgram-" : "-direct-") + ps;
                    c.n = 256; c.window_A = 6.0; c.f = f; c.precision = prec; c.order = order;
                    c.px = c.py = 12; c.n_sites = 9;
                    c.knobs[TUNE_WINDOW_GRAM] = wg; c.knobs[TUNE_RASTER] = 0;
                    if (order == EELS_ORDER_PROBE_FIRST) c.want_wgram = wg ? 1 : 0;
                    cases.push_back(c);
                }
            }
        }
        // raster form: probes on a raster aligned with the f-lattice (step L / (f 64) x 2)
        for (int f : {1, 2}) {
            Case c = mk("");
            c.name = "raster-f" + std::to_string(f) + "-" + ps;
            // the aperture's beams span fewer than 64 lattice columns and rows: L_x f^-1 < 64 / (2 k_ap)
            c.n = f == 1 ? 256 : 512; c.dx = 0.25; c.window_A = 8.0; c.f = f; c.precision = prec;
            c.order = EELS_ORDER_PROBE_FIRST;
            c.px = c.py = 24; c.step = c.n * c.dx / (f * 64.0) * 2; c.n_sites = 7;
            c.knobs[TUNE_RASTER] = 2; c.want_raster = 1;
            cases.push_back(c);
            c.name += "-off-raster";
            c.step *= 1.013;   // off the raster: the plain window-Gram form
            c.want_raster = 0; c.want_wgram = 1; c.knobs[TUNE_WINDOW_GRAM] = 2;
            cases.push_back(c);
        }
        // 256-row tiles of both split GEMMs, stacked Gram rows
        if (prec != EELS_FP32) {
            Case c = mk("");
            c.name = "crop-rows256-" + ps; c.n = 256; c.window_A = 6.0; c.precision = prec;
            c.order = EELS_ORDER_PROBE_FIRST; c.px = c.py = 20; c.knobs[TUNE_GEMM1_ROWS] = 1; c.knobs[TUNE_GEMM2_ROWS] = 1;
            c.knobs[TUNE_WINDOW_GRAM] = 0;
            cases.push_back(c);
            c.name = "crop-rows256-S-" + ps; c.order = EELS_ORDER_S_FIRST; cases.push_back(c);
            Case g = mk("");
            g.name = "full-gram-stack-" + ps; g.precision = prec; g.detsum = EELS_DETSUM_GRAM; g.knobs[TUNE_GRAM_STACK] = 1;
            cases.push_back(g);
        }
        // 384 x 384 grids with crop windows (radix-3 sweeps)
        { Case c = mk(""); c.name = "grid384-crop-" + ps; c.n = 384; c.window_A = 6.0; c.f = 2; c.precision = prec;
          c.px = c.py = 10; cases.push_back(c); }
        { Case c = mk(""); c.name = "grid384-real-space-" + ps; c.n = 384; c.precision = prec; c.real_space = 1;
          c.n_sites = 2; c.trans = 1; c.px = c.py = 4; cases.push_back(c); }
        // slice groups under a budget, resident S-matrices, inverse multislice, companion images
        { Case c = mk(""); c.name = "groups-budget-" + ps; c.n = 256; c.window_A = 6.0; c.nz = 16; c.n_sites = 40;
          c.det_in = 5; c.det_out = 20;
          c.precision = prec; c.tight_budget = true; c.want_groups_gt1 = 1; cases.push_back(c); }
        // window-Gram G epilogue on 256-row Gram tiles (tuning key 10)
        { Case c = mk(""); c.name = "wgram-gram256-" + ps; c.n = 128; c.window_A = 4.0; c.f = 2;
          c.order = EELS_ORDER_PROBE_FIRST; c.precision = prec; c.knobs[TUNE_WINDOW_GRAM] = 2;
          c.knobs[TUNE_GRAM_ROWS] = 1; c.want_wgram = 1; cases.push_back(c); }
        // slice groups resuming from S_1 checkpoints (forced), and under the default rule
        for (double fr : {0.8, 0.6, 0.4}) {
            Case c = mk(""); c.name = "groups-checkpoint-" + std::to_string((int)(100 * fr)) + "-" + ps; c.n = 256;
            c.window_A = 6.0; c.nz = 16; c.n_sites = 800; c.det_in = 5; c.det_out = 20; c.precision = prec;
            c.budget_frac = fr; c.knobs[TUNE_CHECKPOINT] = 2; c.want_groups_gt1 = 1; cases.push_back(c);
            c.name = "groups-checkpoint-rule-" + std::to_string((int)(100 * fr)) + "-" + ps;
            c.knobs[TUNE_CHECKPOINT] = 1; c.want_groups_gt1 = -1; cases.push_back(c);
        }
        { Case c = mk(""); c.name = "resident-" + ps; c.n = 256; c.window_A = 6.0; c.nz = 8; c.n_sites = 12;
          c.precision = prec; c.resident = 1; cases.push_back(c); }
        { Case c = mk(""); c.name = "inverse-" + ps; c.n = 256; c.window_A = 6.0; c.nz = 8; c.n_sites = 10;
          c.precision = prec; c.s1_mode = EELS_S1_INVERSE; cases.push_back(c); }
        { Case c = mk(""); c.name = "s2-retreat-" + ps; c.n = 256; c.window_A = 6.0; c.nz = 8; c.n_sites = 10;
          c.precision = prec; c.s1_mode = EELS_S2_RETREAT; cases.push_back(c); }
        { Case c = mk(""); c.name = "s2-retreat-full-cell-" + ps; c.nz = 4; c.n_sites = 4; c.precision = prec;
          c.s1_mode = EELS_S2_RETREAT; cases.push_back(c); }
        { Case c = mk(""); c.name = "images-" + ps; c.precision = prec; c.n_images = 2; cases.push_back(c); }
    }
    // sizes and probe counts at the edges
    { Case c = mk("grid64-one-probe"); c.n = 64; c.px = c.py = 1; cases.push_back(c); }
    { Case c = mk("grid512-many-probes"); c.n = 512; c.window_A = 8.0; c.f = 2; c.px = c.py = 64; c.n_sites = 20;
      c.precision = EELS_BF16_SPLIT; cases.push_back(c); }
    { Case c = mk("no-sites"); c.n_sites = 0; cases.push_back(c); }
    { Case c = mk("sites-without-transitions"); c.n_sites = 5; c.trans = 1; cases.push_back(c); }
    // invalid problems: each must fail with its status and leave nothing behind
    { Case c = mk("bad-side-100"); c.n = 100; c.expect = EELS_ERR_UNSUPPORTED_SIZE; cases.push_back(c); }
    { Case c = mk("bad-side-2048"); c.n = 2048; c.dx = 0.05; c.expect = EELS_ERR_UNSUPPORTED_SIZE; cases.push_back(c); }
    { Case c = mk("band-basis-384"); c.n = 384; c.expect = EELS_ERR_UNSUPPORTED_SIZE; cases.push_back(c); }
    { Case c = mk("no-probes"); c.px = 0; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }
    { Case c = mk("f-without-window"); c.f = 2; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }
    { Case c = mk("inverse-resident"); c.s1_mode = EELS_S1_INVERSE; c.resident = 1; c.expect = EELS_ERR_INVALID_ARG;
      cases.push_back(c); }
    { Case c = mk("s2-retreat-resident"); c.s1_mode = EELS_S2_RETREAT; c.resident = 1; c.expect = EELS_ERR_INVALID_ARG;
      cases.push_back(c); }
    { Case c = mk("s1-mode-3"); c.s1_mode = 3; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }
    { Case c = mk("images-with-f2"); c.window_A = 6.0; c.n = 256; c.f = 2; c.n_images = 1; c.expect = EELS_ERR_INVALID_ARG;
      cases.push_back(c); }
    { Case c = mk("detector-beyond-band"); c.dx = 0.5; c.expect = EELS_ERR_BANDLIMIT; cases.push_back(c); }
    { Case c = mk("gram-with-f2"); c.window_A = 6.0; c.n = 256; c.f = 2; c.detsum = EELS_DETSUM_GRAM;
      c.precision = EELS_BF16_SPLIT; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }
    { Case c = mk("budget-too-small"); c.budget = 1u << 20; c.expect = EELS_ERR_OOM; cases.push_back(c); }
    { Case c = mk("bad-precision"); c.precision = 7; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }
    { Case c = mk("zero-slices"); c.nz = 0; c.expect = EELS_ERR_INVALID_ARG; cases.push_back(c); }

    for (const Case& c : cases) run_case(c);
    if (g_failures) {
        std::fprintf(stderr, "plan_check: %d failed checks over %zu cases\n", g_failures, cases.size());
        return 1;
    }
    std::printf("plan_check: %zu cases ok (%ld plans: %ld raster, %ld window-Gram, %ld Gram, %ld with slice groups, "
                "%ld with S_1 checkpoints; %ld batches, %ld launched descriptors, %ld reduction entries)\n",
                cases.size(), g_plans, g_raster, g_wgram, g_gram, g_groups, g_ckpt, g_batches, g_descs, g_entries);
    return 0;
}
