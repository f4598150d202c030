// Host planner: validates a problem and lays out every table and buffer the device
// path needs.  Pure host code (no HIP calls), so plans can be built without a GPU.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace eels {

namespace {

constexpr double kH = 6.62607015e-34;       // Planck constant (J s)
constexpr double kM0 = 9.1093837015e-31;    // electron rest mass (kg)
constexpr double kE = 1.602176634e-19;      // elementary charge (C)
constexpr double kC = 299792458.0;          // speed of light (m/s)

// Relativistic wavelength in Angstrom (Sec. 2: lambda of the relativistic electron).
double wavelength_A(double eV) {
    double eE = kE * eV;
    double p = std::sqrt(2.0 * kM0 * eE * (1.0 + eE / (2.0 * kM0 * kC * kC)));
    return kH / p * 1e10;
}

// sigma = 2 pi m e lambda / h^2 with m the relativistic mass, in rad/(V*Angstrom).
double sigma_VA(double eV, double lam_A) {
    double gamma = 1.0 + kE * eV / (kM0 * kC * kC);
    double s = 2.0 * M_PI * gamma * kM0 * kE * (lam_A * 1e-10) / (kH * kH);
    return s * 1e-10;
}

bool pow2_ok(int n) { return n >= 16 && n <= 1024 && (n & (n - 1)) == 0; }
// grid sides of the sweeps: powers of two in [16, 1024], and 384 (= 3 x 128, radix-3 passes)
bool side_ok(int n) { return pow2_ok(n) || n == 384; }

// Plane waves k = (f a / lx, f b / ly) with th_lo <= lambda |k| <= th_hi, ordered by (b, a).
std::vector<int> lattice(double lx, double ly, int f, double lam, double th_lo, double th_hi) {
    int amax = (int)std::floor(th_hi / lam * lx / f) + 1;
    int bmax = (int)std::floor(th_hi / lam * ly / f) + 1;
    std::vector<int> out;
    for (int b = -bmax; b <= bmax; ++b)
        for (int a = -amax; a <= amax; ++a) {
            double kx = (double)(f * a) / lx, ky = (double)(f * b) / ly;
            double th = lam * std::sqrt(kx * kx + ky * ky);
            if (th >= th_lo && th <= th_hi) {
                out.push_back(a);
                out.push_back(b);
            }
        }
    return out;
}

int imod(long long a, int n) { long long r = a % n; return (int)(r < 0 ? r + n : r); }

struct Blob {
    std::vector<int32_t>& v;
    int64_t append(const int32_t* p, size_t n, size_t align_ints = 4) {
        while (v.size() % align_ints) v.push_back(0);
        int64_t off = (int64_t)v.size();
        v.insert(v.end(), p, p + n);
        return off;
    }
    int64_t append(const std::vector<int32_t>& x, size_t align_ints = 4) { return append(x.data(), x.size(), align_ints); }
};

}  // namespace

static eels_status build_plan_impl(Plan& p, const eels_problem& q, size_t blob_reserve) {
    auto fail = [&](eels_status s, const std::string& m) { set_error(m); return s; };
    if (q.nx <= 0 || q.ny <= 0 || !(q.lx_A > 0) || !(q.ly_A > 0) || q.n_slices <= 0 || !q.dz_A)
        return fail(EELS_ERR_INVALID_ARG, "grid, cell or slices invalid");
    if (!side_ok(q.nx) || !side_ok(q.ny))
        return fail(EELS_ERR_UNSUPPORTED_SIZE, "grid sides must be powers of two in [16, 1024] or 384");
    if (q.n_probes <= 0 || !q.probe_xy) return fail(EELS_ERR_INVALID_ARG, "no probes");
    if (q.n_sites < 0 || (q.n_sites > 0 && !q.sites)) return fail(EELS_ERR_INVALID_ARG, "sites");
    if (q.interp_f < 1) return fail(EELS_ERR_INVALID_ARG, "interp_f must be >= 1");
    if (!(q.aperture_mrad > 0) || q.det_inner_mrad < 0 || !(q.det_outer_mrad > q.det_inner_mrad))
        return fail(EELS_ERR_INVALID_ARG, "aperture / detector angles");
    if (q.precision < EELS_FP32 || q.precision > EELS_FP16_SPLIT) return fail(EELS_ERR_INVALID_ARG, "precision");
    if (q.order < EELS_ORDER_AUTO || q.order > EELS_ORDER_PROBE_FIRST) return fail(EELS_ERR_INVALID_ARG, "order");
    if (q.detector_sum < EELS_DETSUM_AUTO || q.detector_sum > EELS_DETSUM_GRAM)
        return fail(EELS_ERR_INVALID_ARG, "detector_sum");
    if (q.s1_mode != EELS_S1_STORED && q.s1_mode != EELS_S1_INVERSE && q.s1_mode != EELS_S2_RETREAT)
        return fail(EELS_ERR_INVALID_ARG, "s1_mode");
    if (q.s1_mode != EELS_S1_STORED && q.resident_s)
        return fail(EELS_ERR_INVALID_ARG, "the inverse multislice keeps no S_1 windows to make resident");
    if (q.n_images < 0 || q.n_images > EELS_MAX_IMAGES || (q.n_images > 0 && !q.image_detectors_mrad))
        return fail(EELS_ERR_INVALID_ARG, "n_images / image_detectors_mrad");
    if (q.n_images > 0 && q.interp_f != 1)
        return fail(EELS_ERR_INVALID_ARG, "companion images need interp_f = 1");
    if (!(q.energy_eV > 0) && !(q.lambda_A > 0 && q.sigma > 0)) return fail(EELS_ERR_INVALID_ARG, "energy");

    p.nx = q.nx; p.ny = q.ny; p.lx = q.lx_A; p.ly = q.ly_A; p.nz = q.n_slices;
    p.dz.assign(q.dz_A, q.dz_A + q.n_slices);
    for (double d : p.dz) if (!(d > 0)) return fail(EELS_ERR_INVALID_ARG, "slice thickness must be > 0");
    p.energy = q.energy_eV;
    p.lam = q.lambda_A > 0 ? q.lambda_A : wavelength_A(q.energy_eV);
    p.sigma = q.sigma > 0 ? q.sigma : sigma_VA(q.energy_eV, p.lam);
    p.alpha = q.aperture_mrad * 1e-3;
    p.beta_in = q.det_inner_mrad * 1e-3;
    p.beta_out = q.det_outer_mrad * 1e-3;
    p.defocus = q.defocus_A; p.cs = q.cs_A;
    p.f = q.interp_f;
    p.bandlimit = q.bandlimit > 0 ? q.bandlimit : 2.0 / 3.0;
    if (p.bandlimit > 1.0) return fail(EELS_ERR_INVALID_ARG, "bandlimit must be <= 1");
    p.window_A = q.window_A;
    p.P = q.n_probes;
    p.probes.assign(q.probe_xy, q.probe_xy + 2 * (size_t)q.n_probes);
    p.sites.assign(q.sites, q.sites + q.n_sites);
    p.n_trans_total = q.n_trans_total;
    p.precision = q.precision;

    // band limit (circular, inclusive) and the kx columns it keeps
    p.kmax = p.bandlimit * std::min(p.nx / (2.0 * p.lx), p.ny / (2.0 * p.ly));
    p.hlx = (int)std::floor(p.kmax * p.lx + 1e-9);
    if (2 * p.hlx + 1 >= p.nx) { p.hlx = p.nx / 2; p.nlx = p.nx; }
    else p.nlx = 2 * p.hlx + 1;
    p.ldx = (int)round_up(p.nlx, 16);   // 128-byte aligned rows of live columns

    // beams
    p.ab1 = lattice(p.lx, p.ly, p.f, p.lam, 0.0, p.alpha);
    p.ab2 = lattice(p.lx, p.ly, p.f, p.lam, p.beta_in, p.beta_out);
    p.N1 = (int)p.ab1.size() / 2;
    p.N2 = (int)p.ab2.size() / 2;
    p.N1fine = (int)lattice(p.lx, p.ly, 1, p.lam, 0.0, p.alpha).size() / 2;
    if (p.N1 == 0 || p.N2 == 0) return fail(EELS_ERR_INVALID_ARG, "empty aperture or detector beam set");
    for (int w = 0; w < 2; ++w) {
        const auto& ab = w == 0 ? p.ab1 : p.ab2;
        for (size_t i = 0; i < ab.size(); i += 2) {
            double kx = (double)(p.f * ab[i]) / p.lx, ky = (double)(p.f * ab[i + 1]) / p.ly;
            if (std::sqrt(kx * kx + ky * ky) > p.kmax)
                return fail(EELS_ERR_BANDLIMIT, w == 0 ? "aperture beyond the band limit" : "detector beyond the band limit");
        }
    }
    p.N1pad = (int)round_up(p.N1, KPAD_MULT);

    // crop window (Sec. 4.B): half-widths floor(W / (2 dx) + 1/2)
    p.full_window = true;
    if (p.window_A > 0) {
        int hx = (int)std::floor(p.window_A / (2.0 * p.lx / p.nx) + 0.5);
        int hy = (int)std::floor(p.window_A / (2.0 * p.ly / p.ny) + 0.5);
        if (2 * hx + 1 < p.nx && 2 * hy + 1 < p.ny) {
            p.full_window = false;
            p.hwx = hx; p.hwy = hy;
        }
    }
    if (p.full_window) { p.nwx = p.nx; p.nwy = p.ny; p.hwx = p.hwy = 0; }
    else { p.nwx = 2 * p.hwx + 1; p.nwy = 2 * p.hwy + 1; }
    p.K = p.nwx * p.nwy;
    p.Kpad = (int)round_up(p.K, KPAD_MULT);
    if (p.f > 1 && p.full_window) return fail(EELS_ERR_INVALID_ARG, "interp_f > 1 needs a crop window");

    // sites: validation, pixels, eligibility
    const int S = (int)p.sites.size();
    p.site_ix0.resize(S); p.site_iy0.resize(S); p.site_probes.assign(S, {});
    const double dx = p.lx / p.nx, dy = p.ly / p.ny;
    for (int s = 0; s < S; ++s) {
        const eels_site& st = p.sites[s];
        if (st.slice < 0 || st.slice >= p.nz || st.n_trans < 0 || st.h_offset < 0 ||
            st.h_offset + st.n_trans > p.n_trans_total)
            return fail(EELS_ERR_INVALID_ARG, "site " + std::to_string(s) + " out of range");
        p.site_ix0[s] = imod((long long)std::floor(st.x_A / (p.lx / p.nx) + 0.5), p.nx);
        p.site_iy0[s] = imod((long long)std::floor(st.y_A / (p.ly / p.ny) + 0.5), p.ny);
        if (p.f > 1) {
            auto& el = p.site_probes[s];
            for (int r = 0; r < p.P; ++r) {
                double ddx = p.site_ix0[s] * dx - p.probes[2 * r];
                double ddy = p.site_iy0[s] * dy - p.probes[2 * r + 1];
                ddx = ddx - p.lx * std::floor(ddx / p.lx + 0.5);
                ddy = ddy - p.ly * std::floor(ddy / p.ly + 0.5);
                if (std::fabs(ddx) + p.hwx * dx <= p.lx / (2.0 * p.f) &&
                    std::fabs(ddy) + p.hwy * dy <= p.ly / (2.0 * p.f))
                    el.push_back(r);
            }
        }
    }
    auto n_elig = [&](int s) { return p.f > 1 ? (int)p.site_probes[s].size() : p.P; };

    // ionised slices and their sites (sites with no transitions or no eligible probe are skipped)
    p.slices.assign(p.nz, SliceInfo{});
    std::vector<std::vector<int>> by_slice(p.nz);
    for (int s = 0; s < S; ++s)
        if (p.sites[s].n_trans > 0 && n_elig(s) > 0) by_slice[p.sites[s].slice].push_back(s);
    std::vector<int> ion;
    for (int j = 0; j < p.nz; ++j)
        if (!by_slice[j].empty()) { ion.push_back(j); p.slices[j].ion = true; }

    // band pixel set of the circular limit |k| <= kmax: live column c keeps |ky index| <= band_h[c]
    p.band_h.assign(p.nlx, -1);
    p.band_off.assign(p.nlx, 0);
    {
        int off = 0;
        for (int c = 0; c < p.nlx; ++c) {
            int cs = p.nlx == p.nx ? (c < (p.nx + 1) / 2 ? c : c - p.nx) : (c <= p.hlx ? c : c - p.nlx);
            double kx = cs / p.lx;
            int h = -1;
            for (int b = 0; b <= p.ny / 2; ++b) {
                double ky = b / p.ly;
                if (std::sqrt(kx * kx + ky * ky) <= p.kmax) h = b;
                else break;
            }
            if (2 * h + 1 > p.ny) h = (p.ny - 1) / 2;
            p.band_h[c] = h;
            p.band_off[c] = off;
            off += std::max(0, 2 * h + 1);
        }
        p.Kb = off;
        p.Kbpad = (int)round_up(std::max(p.Kb, 1), KPAD_MULT);
    }
    // companion-image rings: angles, band-limit check, and the ring bits of every band slot
    p.n_img = q.n_images;
    p.img_in.clear();
    p.img_out.clear();
    std::vector<int32_t> img_mask;
    if (p.n_img > 0) {
        const double band_ang = p.lam * p.kmax;
        for (int d = 0; d < p.n_img; ++d) {
            double a = q.image_detectors_mrad[2 * d] * 1e-3, b = q.image_detectors_mrad[2 * d + 1] * 1e-3;
            if (!(a >= 0) || (b > 0 && !(b > a))) return fail(EELS_ERR_INVALID_ARG, "image detector angles");
            if (b > band_ang * (1 + 1e-12)) return fail(EELS_ERR_BANDLIMIT, "image detector beyond the band limit");
            p.img_in.push_back(a);
            p.img_out.push_back(b > 0 ? b : -1.0);
        }
        img_mask.assign(p.Kbpad, 0);
        for (int c = 0; c < p.nlx; ++c) {
            int cs = p.nlx == p.nx ? (c < (p.nx + 1) / 2 ? c : c - p.nx) : (c <= p.hlx ? c : c - p.nlx);
            int h = p.band_h[c];
            for (int r = 0; r <= 2 * h; ++r) {
                int ks = r <= h ? r : -(2 * h + 1 - r);
                double kx = cs / p.lx, ky = ks / p.ly;
                double th = p.lam * std::sqrt(kx * kx + ky * ky);
                int bits = 0;
                for (int d = 0; d < p.n_img; ++d)
                    if (th >= p.img_in[d] && (p.img_out[d] < 0 || th <= p.img_out[d])) bits |= 1 << d;
                img_mask[p.band_off[c] + r] = bits;
            }
        }
    }
    // full-cell windows contract in the band basis (exact): sum_r S_2 H S_1 equals the sum
    // over band pixels g of (P_j x_{j+1})(g) * fft2(T_j H S_1)(g)
    // (the S_2 retreat captures real-space windows only: its plans always contract in real space)
    p.recip = p.full_window && !q.real_space && q.s1_mode != EELS_S2_RETREAT;
    if (p.recip && (!pow2_ok(p.nx) || !pow2_ok(p.ny)))
        return fail(EELS_ERR_UNSUPPORTED_SIZE, "the band-basis contraction needs power-of-two grid sides "
                                               "(use a crop window or real_space)");
    const bool split = p.precision != EELS_FP32;
    const int Kc = p.recip ? p.Kb : p.K;            // contraction length of the big GEMM
    const int Kcpad = p.recip ? p.Kbpad : p.Kpad;

    // Gram form of the detector sum: every probe must cover every site (f = 1), and the
    // first product must not carry H in its prologue (FP32 real-space contraction)
    const bool gram_ok = p.f == 1 && (p.recip || split) && q.order != EELS_ORDER_PROBE_FIRST;
    if (q.detector_sum == EELS_DETSUM_GRAM && !gram_ok)
        return fail(EELS_ERR_INVALID_ARG, "the Gram detector sum needs interp_f = 1, order S and the band basis "
                                          "or a split precision");
    const bool want_gram = gram_ok && q.detector_sum != EELS_DETSUM_DIRECT;

    // contraction order (Eq. TPRISM2 terms; both orders compute the same sums).  Gram form:
    // the Hermitian half of each site's Z^H Z plus one quadratic form per probe.
    double fl_S = 0, fl_P = 0, fl_G = 0, fl_D = 0, fl_W = 0;
    for (int j : ion)
        for (int s : by_slice[j]) {
            double nt = p.sites[s].n_trans, Ps = n_elig(s);
            // order P's second product: per transition (S_2w H_n) Psi, or in the window-Gram
            // form the Hermitian half of S_2w^H S_2w plus G Psi
            fl_D += 8.0 * p.N2 * (double)Kc * nt * Ps;
            fl_W += 4.0 * p.N2 * (double)Kc * (Kc + 1.0) + 8.0 * Ps * (double)Kc * Kc;
            double g1 = 8.0 * p.N2 * (double)Kc * nt * p.N1;
            fl_S += g1 + 8.0 * nt * p.N2 * p.N1 * Ps;
            fl_G += g1 + 8.0 * nt * p.N2 * 0.5 * p.N1 * (p.N1 + 1.0);
            fl_P += 8.0 * Ps * (double)p.K * p.N1 + 8.0 * p.N2 * (double)Kc * nt * Ps;
        }
    if (!ion.empty()) fl_G += 8.0 * p.N1 * (double)p.N1 * p.P;
    if (want_gram) fl_S = std::min(fl_S, fl_G);
    if (q.order != EELS_ORDER_AUTO) p.order = q.order;
    else if (q.detector_sum == EELS_DETSUM_GRAM) p.order = EELS_ORDER_S_FIRST;   // the Gram form is order S
    else p.order = fl_S <= fl_P ? EELS_ORDER_S_FIRST : EELS_ORDER_PROBE_FIRST;
    p.gram = want_gram && p.order == EELS_ORDER_S_FIRST &&
             (q.detector_sum == EELS_DETSUM_GRAM || fl_G <= fl_S);
    p.N2p = (int)round_up(p.N2, KPAD_MULT);
    p.gemm_flops = p.order == EELS_ORDER_S_FIRST ? (p.gram ? fl_G : fl_S) : fl_P;
    p.c_scale = p.precision == EELS_FP16_SPLIT ? 256.0f : 1.0f;
    const bool orderS = p.order == EELS_ORDER_S_FIRST;
    p.c_sc = (split && !p.gram) ? p.precision : 0;   // the Gram quadratic form reads complex64
    // order P in split precision with cropped windows: A_n = (S_2w H_n) Psi, so the producer
    // writes n_t x N_2 window rows instead of n_t x P_s probe rows (N_2 < P_s on large scans)
    // and reads the S_2 windows captured in complex64
    p.hs2 = split && !orderS && !p.recip;
    // window-Gram form (plan-time knob 6): I(R) = f^2 Psi_R^H (M o sum_t conj(H_t) H_t^T) Psi_R
    // with M = S_2w^H S_2w, one Gram GEMM per site instead of n_t products with N_2 rows
    const int wg_knob = tune_get(TUNE_WINDOW_GRAM);    // 0 never, 1 with fewer flops, 2 wherever it applies
    // (FP32 too: an FP32 Gram GEMM, G in complex64 and an FP32 G Psi product)
    p.wgram = !orderS && !p.recip && !p.full_window && p.Kpad <= 4096 &&
              (wg_knob == 2 || (wg_knob == 1 && fl_W < fl_D));
    // raster form of the window-Gram detector sum (plan-time knob 7: 0 never, 1 where it needs
    // fewer flops, 2 wherever it applies).  When every probe sits on a raster aligned with the
    // beam lattice, R = R_0 + (i L_x / (f M), j L_y / (f M)) with integers i, j, the probe phase
    // exp(-2 pi i k.R) is exp(-2 pi i k.R_0) times the M x M DFT kernel exp(-2 pi i (a i + b j) / M)
    // of the beam's lattice coordinates (a, b).  Psi(R, r) = sum_k c_k(R) S_1[k](r) for every
    // probe is then one 2-D DFT per window pixel, and so is Y(R, r) = sum_r' G(r, r') Psi(R, r')
    // from Z = G S_1w^T (K^2 N_1 GEMM flops instead of K N_1 P_s + K^2 P_s).  The DFT does not
    // alias when the beams' a and b each span fewer than M values.
    {
        const int r_knob = tune_get(TUNE_RASTER);
        const int M = 64;
        p.raster = false;
        if (!orderS && !p.recip && !p.full_window && p.Kpad <= 4096 && r_knob != 0 && wg_knob != 0) {
            int amin = 1 << 30, amax = -(1 << 30), bmin = 1 << 30, bmax = -(1 << 30);
            for (int b = 0; b < p.N1; ++b) {
                amin = std::min(amin, p.ab1[2 * b]); amax = std::max(amax, p.ab1[2 * b]);
                bmin = std::min(bmin, p.ab1[2 * b + 1]); bmax = std::max(bmax, p.ab1[2 * b + 1]);
            }
            bool ok = amax - amin < M && bmax - bmin < M;
            std::vector<int> res(p.P);
            for (int r = 0; ok && r < p.P; ++r) {
                const double u = (p.probes[2 * r] - p.probes[0]) * p.f / p.lx * M;
                const double v = (p.probes[2 * r + 1] - p.probes[1]) * p.f / p.ly * M;
                const double ru = std::nearbyint(u), rv = std::nearbyint(v);
                if (std::fabs(u - ru) > 1e-6 || std::fabs(v - rv) > 1e-6) ok = false;
                else res[r] = imod((long long)ru, M) + M * imod((long long)rv, M);
            }
            double fl_R = 0;
            for (int j : ion)
                for (size_t t = 0; t < by_slice[j].size(); ++t)
                    fl_R += 4.0 * p.N2 * (double)p.K * (p.K + 1.0) + 8.0 * (double)p.K * p.K * p.N1;
            const double fl_cur = p.wgram ? fl_P - fl_D + fl_W : fl_P;
            if (ok && (r_knob == 2 || fl_R < fl_cur)) {
                p.raster = true;
                p.wgram = true;
                p.rM = M;
                p.r_res = std::move(res);
                p.r_chunk = 64;
                p.r_chunks = (int)ceil_div(p.K, p.r_chunk);
            }
        }
    }
    // split window-Gram form: G from the Gram GEMM's epilogue (tuning key 9: 1 where every site
    // has at most 32 transitions, 0 never: the Gram tiles M and a separate combine kernel)
    {
        int max_nt = 0;
        for (const auto& st : p.sites) max_nt = std::max(max_nt, st.n_trans);
        p.wg_fused = split && p.wgram && max_nt <= 32 && tune_get(TUNE_WG_FUSED) != 0;
    }
    p.w2_sc = (split && !p.hs2) ? p.precision : 0;
    p.mid2_sc = split ? p.precision : 0;

    // windows per slice
    auto slice_windows = [&](int j) -> int { return p.full_window ? 1 : (int)by_slice[j].size(); };
    int max_w2 = 0;
    for (int j : ion) max_w2 = std::max(max_w2, slice_windows(j));
    p.max_w2 = max_w2;
    const int64_t w2_slice = p.recip ? (int64_t)p.N2 * p.Kbpad : (int64_t)max_w2 * p.N2 * p.Kpad;
    p.resident = q.resident_s != 0;
    // raster form in split precision: the S_1 capture writes the windows SC with each beam's
    // c_k(R_0) folded in, so they are the Z product's operand as they stand (resident windows
    // serve new probes, whose c_k(R_0) differ, and keep complex64)
    p.w1_sc = (p.raster && split && !p.resident) ? p.precision : 0;
    p.slice_w2.assign(p.nz, 0);
    int64_t w2_elems = w2_slice;
    if (p.resident) {
        int64_t off = 0;
        for (int j : ion) { p.slice_w2[j] = off; off += w2_slice; }
        w2_elems = std::max<int64_t>(off, 1);
    }

    // per-site intermediates: mid (Z or Psi), mid2 (H-multiplied operand, split or band
    // basis), band-FFT scratch, norm partial sums
    auto site_mid = [&](int s) -> int64_t {
        int nt = p.sites[s].n_trans;
        if (p.gram) return (int64_t)p.N1 * nt * p.N2p;     // Z rows [t k][q]
        if (p.raster) return 0;                            // no Psi is stored
        return orderS ? (int64_t)nt * p.N2 * p.N1pad : (int64_t)n_elig(s) * p.Kpad;
    };
    auto site_ni = [&](int s) -> int64_t { return orderS ? p.N1 : (p.hs2 ? p.N2 : n_elig(s)); };
    // window-Gram layout of a site's mid2 region (complex units): S_2w transposed [K][N_2p],
    // M [K][Kpad] (FP32 complex), G [K][Kpad], Y^T [P_s][Kpad]
    const int64_t wg_m = (int64_t)p.K * p.N2p, wg_g = wg_m + (int64_t)p.K * p.Kpad,
                  wg_y = wg_g + (int64_t)p.K * p.Kpad;
    auto site_mid2 = [&](int s) -> int64_t {
        if (!p.recip && !split && !p.wgram) return 0;
        // raster form: Z [K][N_1p] at wg_y, then Xt [K][N_1p], then (split, windows not captured
        // SC) S_1w as SC [N_1][Kpad]
        int64_t m2 = p.raster ? wg_y + 2 * (int64_t)p.K * p.N1pad + (split && !p.w1_sc ? (int64_t)p.N1 * p.Kpad : 0)
                   : p.wgram ? wg_y + (int64_t)n_elig(s) * p.Kpad
                             : (int64_t)p.sites[s].n_trans * site_ni(s) * Kcpad;
        // order P, split: the site's S_1 window is first transposed here for the product C S_1w
        if (split && !orderS) m2 = std::max(m2, (int64_t)p.K * p.N1pad);
        return m2;
    };
    auto site_part = [&](int s) -> int64_t {
        if (p.gram) return 2 * (int64_t)p.sites[s].n_trans * p.N1pad * p.N1pad;   // FP32 partials of Z_t^H Z_t
        if (p.raster) return (int64_t)p.r_chunks * p.rM * p.rM;                  // one per residue and DFT block
        if (p.wgram) return n_elig(s);                                            // one per eligible probe
        int nt = p.sites[s].n_trans;
        int64_t tm = ceil_div(p.N2, GEMM_BM);
        return tm * nt * (int64_t)n_elig(s);
    };
    int64_t scratch = 0;
    if (p.recip)
        for (int j : ion)
            for (int s : by_slice[j])
                scratch = std::max(scratch, (int64_t)p.sites[s].n_trans * site_ni(s) * p.ny * p.ldx);
    p.scratch_elems = scratch;

    // fixed workspace
    auto A = [](size_t x) { return (size_t)round_up((int64_t)x, 256); };
    const size_t c8 = 8;  // bytes per complex64
    size_t fixed = A(blob_reserve)  // table blob (refined by the caller's second pass)
                   + A(c8 * p.nx) + A(c8 * p.ny) + A(c8 * (size_t)p.nz * p.ny * p.nx) +
                   A(c8 * (size_t)p.nz * (p.nlx + p.ny)) + A(c8 * (size_t)p.P * p.N1pad) +
                   A(c8 * (size_t)p.N1 * p.ny * p.ldx) + A(c8 * (size_t)p.N2 * p.ny * p.ldx) +
                   A(c8 * (size_t)w2_elems) + A(c8 * (size_t)scratch) +
                   (p.gram ? A(16 * (size_t)p.N1 * p.N1) + A(8 * (size_t)p.P * ceil_div(p.N1, 64)) : 0) +
                   (p.raster ? A(c8 * (size_t)p.N1pad) + A(c8 * (size_t)p.rM) : 0) +
                   (p.n_img > 0 ? 2 * A(c8 * (size_t)p.N1 * p.Kbpad) + A(c8 * (size_t)p.N1pad * p.N1pad) +
                                      A(16 * (size_t)p.N1 * p.N1) + A(8 * (size_t)p.P * ceil_div(p.N1, 64)) +
                                      A(c8 * (size_t)p.P * p.N1pad)
                                : 0);

    size_t budget = q.max_workspace_bytes;
    size_t batch_cap = SIZE_MAX;
    const size_t win1_bytes = c8 * (size_t)p.N1 * p.Kpad;
    if (budget > 0) {
        if (budget <= fixed) return fail(EELS_ERR_OOM, "memory budget below the fixed workspace");
        // at least one slice's S_1 windows must fit next to the contraction buffers;
        // the contraction batches get half of what remains beyond that, a quarter in the
        // window-Gram form (its per-site buffers are smaller, and the room left to the S_1
        // windows means fewer slice groups, each of which reruns the forward sweep)
        size_t min_w1 = 0;
        for (int j : ion) min_w1 = std::max(min_w1, (size_t)slice_windows(j) * win1_bytes);
        size_t avail = budget - fixed;
        if (avail <= min_w1 + 4096) return fail(EELS_ERR_OOM, "memory budget too small for one slice's windows");
        batch_cap = (avail - min_w1 - 4096) / (p.wgram ? 4 : 2);
    }
    struct PendingBatch { int slice; std::vector<int> sites; };
    std::vector<PendingBatch> pend;
    int64_t max_mid = 0, max_mid2 = 0, max_part = 0;
    for (int j : ion) {
        PendingBatch cur{j, {}};
        int64_t m = 0, m2 = 0, pt = 0;
        for (int s : by_slice[j]) {
            int64_t sm = site_mid(s), sm2 = site_mid2(s), sp = site_part(s);
            size_t bytes_new = (size_t)(m + sm + m2 + sm2) * 8 + (size_t)(pt + sp) * 4;
            if (!cur.sites.empty() && bytes_new > batch_cap) {
                pend.push_back(cur);
                max_mid = std::max(max_mid, m); max_mid2 = std::max(max_mid2, m2); max_part = std::max(max_part, pt);
                cur.sites.clear(); m = 0; m2 = 0; pt = 0;
            }
            if ((size_t)(sm + sm2) * 8 + (size_t)sp * 4 > batch_cap)
                return fail(EELS_ERR_OOM, "one site's contraction does not fit the budget");
            cur.sites.push_back(s); m += sm; m2 += sm2; pt += sp;
        }
        pend.push_back(cur);
        max_mid = std::max(max_mid, m); max_mid2 = std::max(max_mid2, m2); max_part = std::max(max_part, pt);
    }
    p.mid_elems = max_mid;
    p.mid2_elems = max_mid2;
    p.part_elems = max_part;

    // slice groups (descending): S_1 windows of a group must fit what is left
    size_t w1_cap = SIZE_MAX;
    if (budget > 0) {
        size_t used = fixed + A((size_t)max_mid * 8) + A((size_t)max_mid2 * 8) + A((size_t)max_part * 4);
        if (budget <= used) return fail(EELS_ERR_OOM, "memory budget too small");
        w1_cap = budget - used;
    }
    p.groups.clear();
    p.site_w1.assign(S, -1);
    p.site_w2.assign(S, -1);
    p.s1_inverse = q.s1_mode == EELS_S1_INVERSE;
    p.s2_retreat = q.s1_mode == EELS_S2_RETREAT;
    if (p.s1_inverse || p.s2_retreat) {
        // one pass; the windows of one slice at a time
        int maxw = 0;
        for (int j : ion) {
            if ((size_t)slice_windows(j) * win1_bytes > w1_cap)
                return fail(EELS_ERR_OOM, "one slice's S_1 windows exceed the budget");
            p.slices[j].group = 0;
            if (p.full_window) for (int s : by_slice[j]) p.site_w1[s] = 0;
            else for (size_t t = 0; t < by_slice[j].size(); ++t) p.site_w1[by_slice[j][t]] = (int)t;
            maxw = std::max(maxw, slice_windows(j));
        }
        if (!ion.empty()) p.groups.push_back(Group{ion.front(), ion.back(), maxw});
    } else {
        // Groups from the top ionised slice down, each holding as many slices' S_1 windows as
        // w1_cap allows; (j_hi, j_lo) per group.
        auto form = [&](size_t cap, std::vector<std::pair<int, int>>& gr) -> bool {
            gr.clear();
            size_t gbytes = 0;
            for (int idx = (int)ion.size() - 1; idx >= 0; --idx) {
                const int j = ion[idx];
                const size_t need = (size_t)slice_windows(j) * win1_bytes;
                if (need > cap) return false;
                if (gr.empty() || gbytes + need > cap) {
                    gr.push_back({j, j});
                    gbytes = 0;
                }
                gr.back().second = j;
                gbytes += need;
            }
            return true;
        };
        // Forward-sweep cost in beam-slice passes: without a checkpoint a group sweeps S_1 from
        // slice 0 to its top slice; with one, a group after the first resumes from S_1 at the
        // entrance of its lowest slice, saved while the first group's sweep passed it (two copies
        // of the state, counted as one pass), which saves j_lo - 1 passes.
        auto cost = [&](const std::vector<std::pair<int, int>>& g, const std::vector<char>& ck) {
            double c = 0;
            for (size_t k = 0; k < g.size(); ++k) c += ck[k] ? g[k].first - g[k].second + 2 : g[k].first + 1;
            return c;
        };
        // n slots go to the n later groups whose lowest slice is highest (the largest savings)
        auto assign = [&](const std::vector<std::pair<int, int>>& g, size_t n, std::vector<char>& ck) {
            ck.assign(g.size(), 0);
            std::vector<size_t> cand;
            for (size_t k = 1; k < g.size(); ++k)
                if (g[k].second > 1) cand.push_back(k);
            std::sort(cand.begin(), cand.end(), [&](size_t a, size_t b) { return g[a].second > g[b].second; });
            for (size_t i = 0; i < cand.size() && i < n; ++i) ck[cand[i]] = 1;
        };
        std::vector<std::pair<int, int>> gr, grk;
        std::vector<char> ck, ckk;
        if (!form(w1_cap, gr)) return fail(EELS_ERR_OOM, "one slice's S_1 windows exceed the budget");
        ck.assign(gr.size(), 0);
        // S_1 checkpoints (tuning key 8: 0 never, 1 where the sweeps cost less, 2 whenever there
        // are several groups): n slots take n ckpt_bytes from the windows' share, so the groups
        // are formed again for each n; the n of the lowest cost is taken
        const int ck_knob = tune_get(TUNE_CHECKPOINT);
        const size_t ckpt_bytes = A(c8 * (size_t)p.N1 * p.ny * p.ldx);
        if (gr.size() > 1 && ck_knob != 0 && budget > 0 && !p.resident) {
            double best = ck_knob == 2 ? 1e300 : cost(gr, ck);
            std::vector<std::pair<int, int>> keep_gr = gr;
            for (size_t n = 1; n <= ion.size() && n * ckpt_bytes < w1_cap; ++n) {
                if (!form(w1_cap - n * ckpt_bytes, grk)) break;
                assign(grk, n, ckk);
                if (std::count(ckk.begin(), ckk.end(), 1) < (long)n) break;   // more slots than groups to use them
                const double c = cost(grk, ckk);
                if (c < best) { best = c; keep_gr = grk; ck = ckk; }
            }
            gr = keep_gr;
            if (ck.size() != gr.size()) ck.assign(gr.size(), 0);
        }
        p.n_ckpt = 0;
        for (size_t gi = 0; gi < gr.size(); ++gi) {
            Group g{gr[gi].second, gr[gi].first, 0};
            if (ck[gi]) {
                g.ckpt = p.n_ckpt++;
                p.slices[g.j_lo].ckpt_save = g.ckpt;
            }
            int gwin = 0;
            for (int idx = (int)ion.size() - 1; idx >= 0; --idx) {
                const int j = ion[idx];
                if (j > g.j_hi || j < g.j_lo) continue;
                p.slices[j].group = (int)gi;
                if (p.full_window) {
                    for (int s : by_slice[j]) p.site_w1[s] = gwin;
                    gwin += 1;
                } else {
                    for (size_t t = 0; t < by_slice[j].size(); ++t) p.site_w1[by_slice[j][t]] = gwin + (int)t;
                    gwin += (int)by_slice[j].size();
                }
            }
            g.n_windows = gwin;
            p.groups.push_back(g);
        }
    }
    if (p.resident && p.groups.size() > 1)
        return fail(EELS_ERR_OOM, "resident S-matrices need every S_1 window in one slice group");
    p.max_w1 = 0;
    for (auto& g : p.groups) p.max_w1 = std::max(p.max_w1, g.n_windows);
    for (int j : ion) {
        const auto& v = by_slice[j];
        for (size_t t = 0; t < v.size(); ++t) p.site_w2[v[t]] = p.full_window ? 0 : (int)t;
    }

    // ---- table blob
    p.blob.clear();
    Blob B{p.blob};
    auto live_col = [&](int ix) -> int {
        if (p.nlx == p.nx) return ix;
        if (ix <= p.hlx) return ix;
        return ix - p.nx + p.nlx;
    };
    {
        std::vector<int32_t> t;
        for (int b = 0; b < p.N1; ++b) {
            int a = p.ab1[2 * b], bb = p.ab1[2 * b + 1];
            t.push_back(live_col(imod((long long)p.f * a, p.nx)));
            t.push_back(imod((long long)p.f * bb, p.ny));
            t.push_back(a); t.push_back(bb);
        }
        p.b1_off = B.append(t);
        t.clear();
        for (int b = 0; b < p.N2; ++b) {
            int a = p.ab2[2 * b], bb = p.ab2[2 * b + 1];
            t.push_back(live_col(imod((long long)p.f * a, p.nx)));
            t.push_back(imod((long long)p.f * bb, p.ny));
            t.push_back(a); t.push_back(bb);
        }
        p.b2_off = B.append(t);
        t.resize(p.P);
        for (int r = 0; r < p.P; ++r) t[r] = r;
        p.ident_off = B.append(t);
        p.band_h_off = B.append(std::vector<int32_t>(p.band_h.begin(), p.band_h.end()));
        p.band_off_off = B.append(std::vector<int32_t>(p.band_off.begin(), p.band_off.end()));
    }
    // capture CSRs per ionised slice (S_2 windows only in the real-space contraction)
    for (int j : ion) {
        for (int which = 0; which < 2; ++which) {
            if (which == 1 && p.recip) continue;
            std::vector<std::vector<CaptureRec>> rows(p.ny);
            if (p.full_window) {
                int w = which == 0 ? p.site_w1[by_slice[j][0]] : 0;
                for (int y = 0; y < p.ny; ++y) rows[y].push_back(CaptureRec{w, y, 0, p.nx});
            } else {
                for (int s : by_slice[j]) {
                    int w = which == 0 ? p.site_w1[s] : p.site_w2[s];
                    for (int v = 0; v < p.nwy; ++v) {
                        int y = imod((long long)p.site_iy0[s] - p.hwy + v, p.ny);
                        rows[y].push_back(CaptureRec{w, v, imod((long long)p.site_ix0[s] - p.hwx, p.nx), p.nwx});
                    }
                }
            }
            std::vector<int32_t> ptr(p.ny + 1, 0), rec;
            for (int y = 0; y < p.ny; ++y) {
                for (auto& r : rows[y]) { rec.push_back(r.win); rec.push_back(r.dy); rec.push_back(r.x0); rec.push_back(r.nwx); }
                ptr[y + 1] = (int32_t)(rec.size() / 4);
            }
            int64_t po = B.append(ptr), ro = B.append(rec);
            if (which == 0) { p.slices[j].cap1_ptr = po; p.slices[j].cap1_rec = ro; }
            else { p.slices[j].cap2_ptr = po; p.slices[j].cap2_rec = ro; }
        }
    }
    // eligible-probe lists
    std::vector<int64_t> site_idx(S, -1);
    for (int s = 0; s < S; ++s) {
        if (p.f > 1 && !p.site_probes[s].empty())
            site_idx[s] = B.append(std::vector<int32_t>(p.site_probes[s].begin(), p.site_probes[s].end()));
        else site_idx[s] = p.ident_off;
    }
    // raster form: the beams in the order the DFT block's threads read them (thread 4 y + x mod 4
    // holds grid slot (x, y) = (a mod M, b mod M) in register x / 4, and consecutive threads of
    // one register read consecutive columns), and each grid slot's column (-1: no beam)
    if (p.raster) {
        const int M = p.rM;
        std::vector<std::pair<int, int>> key(p.N1);
        std::vector<int> slot(p.N1);
        for (int b = 0; b < p.N1; ++b) {
            const int x = imod(p.ab1[2 * b], M), y = imod(p.ab1[2 * b + 1], M);
            slot[b] = y * M + x;
            key[b] = {(x >> 2) * 4 * M + 4 * y + (x & 3), b};
        }
        std::sort(key.begin(), key.end());
        std::vector<int32_t> perm(p.N1), pos((size_t)M * M, -1);
        for (int q = 0; q < p.N1; ++q) {
            perm[q] = key[q].second;
            if (pos[slot[key[q].second]] >= 0) return fail(EELS_ERR_INTERNAL, "two beams on one DFT slot");
            pos[slot[key[q].second]] = q;
        }
        p.r_perm_off = B.append(perm);
        p.r_pos_off = B.append(pos);
    }
    // descriptors, producer jobs and reduction CSRs
    p.descs.clear();
    p.batches.clear();
    p.jobs.clear();
    const int64_t w1_stride = (int64_t)p.N1 * p.Kpad, w2_stride = (int64_t)p.N2 * p.Kpad;
    const bool h_in_gemm = !p.recip && !split;     // FP32 real-space: H applied in the GEMM prologue
    const bool gram_stack = tune_get(TUNE_GRAM_STACK) != 0;
    // the split first GEMM (a store epilogue in both orders) may use 256-row tiles
    const int rows1 = (split && tune_get(TUNE_GEMM1_ROWS) != 0) ? 256 : GEMM_BM;
    // and so may the split second GEMM with the norm epilogue (not the Gram tiles)
    const int rows2 = (split && !p.gram && tune_get(TUNE_GEMM2_ROWS) != 0) ? 256 : GEMM_BM;
    for (auto& pb : pend) {
        Batch bt{};
        bt.slice = pb.slice;
        bt.order = p.order;
        int64_t moff = 0, m2off = 0, poff = 0;
        std::vector<int64_t> site_moff, site_m2off;
        for (int s : pb.sites) {
            site_moff.push_back(moff); site_m2off.push_back(m2off);
            moff += site_mid(s); m2off += site_mid2(s);
        }
        // producer jobs (band FFT or H multiply) write mid2 from S_1 windows (order S) or Psi (order P)
        bt.job_begin = (int)p.jobs.size();
        if (p.recip || split || p.wgram) {
            for (size_t si = 0; si < pb.sites.size(); ++si) {
                int s = pb.sites[si];
                Job jb{};
                jb.from_mid = orderS ? 0 : (p.hs2 ? 2 : 1);
                jb.w_off = orderS ? (int64_t)p.site_w1[s] * w1_stride
                                  : ((p.hs2 || p.wgram) ? p.slice_w2[pb.slice] + (int64_t)p.site_w2[s] * w2_stride
                                                        : site_moff[si]);
                jb.win_off = (int64_t)p.site_w1[s] * w1_stride;
                jb.Ni = (int)site_ni(s);
                jb.nt = p.sites[s].n_trans;
                jb.h_off = p.sites[s].h_offset * p.K;
                jb.dst_off = site_m2off[si];
                if (p.wgram) {
                    jb.s2t_off = site_m2off[si];
                    jb.m_off = site_m2off[si] + wg_m;
                    jb.g_off = site_m2off[si] + wg_g;
                    jb.y_off = site_m2off[si] + wg_y;
                    jb.psi_off = site_moff[si];
                    jb.ps = n_elig(s);
                    if (p.raster) {
                        jb.xt_off = jb.y_off + (int64_t)p.K * p.N1pad;
                        jb.s1sc_off = jb.xt_off + (int64_t)p.K * p.N1pad;
                    }
                }
                p.jobs.push_back(jb);
            }
        }
        bt.job_count = (int)p.jobs.size() - bt.job_begin;

        bt.d1_begin = (int)p.descs.size();
        int tiles = 0;
        for (size_t si = 0; si < pb.sites.size() && !p.raster; ++si) {
            int s = pb.sites[si];
            const eels_site& st = p.sites[s];
            int Ps = n_elig(s);
            GemmDesc d{};
            if (orderS && p.gram) {
                // Z_s[t k][q] = sum_r (H_t S1w)[k][r] S2w[q][r]  (or its band-basis form): the
                // transitions' rows stacked into one M = n_t N_1 (S_2 is shared, and the
                // stacked rows fill the 128-row tiles), or one problem per transition
                d.a_off = site_m2off[si]; d.lda = Kcpad;
                if (p.recip) { d.b_off = p.slice_w2[pb.slice]; d.ldb = p.Kbpad; }
                else { d.b_off = p.slice_w2[pb.slice] + (int64_t)p.site_w2[s] * w2_stride; d.ldb = p.Kpad; }
                d.b_tstride = 0;
                d.h_off = -1;
                d.c_off = site_moff[si]; d.ldc_m = p.N2p;
                if (gram_stack) {
                    d.a_tstride = 0; d.ldc_t = 0;
                    d.M = st.n_trans * p.N1; d.n_t = 1;
                } else {
                    d.a_tstride = (int64_t)p.N1 * Kcpad; d.ldc_t = (int64_t)p.N1 * p.N2p;
                    d.M = p.N1; d.n_t = st.n_trans;
                }
                d.N_inner = p.N2; d.K = Kc;
                d.idx_off = -1;
                d.flags = GD_ZERO_PAD;
            } else if (orderS) {
                // Z_s[t][q][k] = sum_r S2w[q][r] H_t[r] S1w[k][r]  (or its band-basis form)
                if (p.recip) { d.a_off = p.slice_w2[pb.slice]; d.lda = p.Kbpad; }
                else { d.a_off = p.slice_w2[pb.slice] + (int64_t)p.site_w2[s] * w2_stride; d.lda = p.Kpad; }
                if (h_in_gemm) {
                    d.b_off = (int64_t)p.site_w1[s] * w1_stride; d.ldb = p.Kpad;
                    d.h_off = st.h_offset * p.K; d.ldh = p.K;
                } else {
                    d.b_off = site_m2off[si]; d.ldb = Kcpad; d.b_tstride = (int64_t)p.N1 * Kcpad;
                    d.h_off = -1;
                }
                d.c_off = site_moff[si]; d.ldc_m = p.N1pad; d.ldc_t = (int64_t)p.N2 * p.N1pad;
                d.M = p.N2; d.N_inner = p.N1; d.n_t = st.n_trans; d.K = Kc;
                d.idx_off = -1;
            } else {
                // Psi_s[i][r] = sum_k C[idx[i]][k] S1w[k][r]: FP32 reads S1w as an N-contiguous
                // B operand; split reads the SC transpose of the window written into mid2
                d.a_off = 0; d.lda = p.N1pad;
                if (split) {
                    d.b_off = site_m2off[si]; d.ldb = p.N1pad;
                    d.flags = GD_IDX_A;
                } else {
                    d.b_off = (int64_t)p.site_w1[s] * w1_stride; d.ldb = p.Kpad;
                }
                d.h_off = -1; d.ldh = 0;
                d.c_off = site_moff[si]; d.ldc_m = p.Kpad; d.ldc_t = 0;
                d.M = Ps; d.N_inner = p.K; d.n_t = 1; d.K = p.N1;
                d.idx_off = site_idx[s];
            }
            d.tiles_m = (int)ceil_div(d.M, rows1);
            d.tiles_n = (int)ceil_div(d.N_inner, GEMM_BN);
            d.tile_start = tiles;
            tiles += d.tiles_m * d.tiles_n * d.n_t;
            p.descs.push_back(d);
        }
        bt.d1_count = (int)p.descs.size() - bt.d1_begin;
        bt.d1_tiles = tiles;
        bt.d1_rows = rows1;
        // second GEMM
        bt.d2_begin = (int)p.descs.size();
        tiles = 0;
        std::vector<std::vector<int32_t>> ent(p.P);
        for (size_t si = 0; si < pb.sites.size(); ++si) {
            int s = pb.sites[si];
            const eels_site& st = p.sites[s];
            int Ps = n_elig(s);
            const std::vector<int>* pl = p.f > 1 ? &p.site_probes[s] : nullptr;
            GemmDesc d{};
            if (orderS && p.gram) {
                // G_t[k][k'] = sum_q conj(Z_s[t k][q]) Z_s[t k'][q]  (upper tiles), one FP32
                // partial per transition; the partials are summed in FP64
                d.a_off = site_moff[si]; d.lda = p.N2p; d.a_tstride = (int64_t)p.N1 * p.N2p;
                d.b_off = site_moff[si]; d.ldb = d.lda; d.b_tstride = d.a_tstride;
                d.h_off = -1; d.ldh = 0;
                d.c_off = 0; d.ldc_m = p.N1pad; d.ldc_t = (int64_t)p.N1pad * p.N1pad;
                d.M = p.N1; d.N_inner = p.N1; d.n_t = st.n_trans; d.K = p.N2p;
                d.idx_off = -1;
                d.tiles_m = (int)ceil_div(d.M, GEMM_BM);
                d.tiles_n = (int)ceil_div(d.N_inner, GEMM_BN);
                d.tile_start = tiles;
                d.p_off = poff; d.ld_part = 0;     // float2 offset of the site's first partial
                poff += (int64_t)st.n_trans * p.N1pad * p.N1pad;
                tiles += d.tiles_m * d.tiles_n * d.n_t;
                bt.n_parts += st.n_trans;
                p.descs.push_back(d);
                continue;
            }
            if (p.wgram) {
                // the site's per-probe results of the window-Gram form, one FP32 partial per
                // eligible probe (this descriptor only drives the reduction)
                d.h_off = -1; d.idx_off = -1;
                d.M = 0; d.N_inner = Ps; d.n_t = 1; d.K = 0;
                d.tiles_m = 1; d.tiles_n = 0; d.tile_start = tiles;
                d.p_off = poff; d.ld_part = Ps;
                if (p.raster) {
                    // the site's DFT blocks each leave M^2 partial sums, one per probe residue;
                    // a probe's entry is its residue and the reduction adds the blocks' values
                    d.N_inner = p.rM * p.rM;
                    d.tiles_m = p.r_chunks;
                    d.ld_part = (int64_t)p.rM * p.rM;
                }
                p.jobs[bt.job_begin + si].part_off = poff;
                poff += d.tiles_m * d.ld_part;
                int di = (int)p.descs.size();
                p.descs.push_back(d);
                if (p.f > 1 || p.raster)
                    for (int i = 0; i < Ps; ++i) {
                        int r = pl ? (*pl)[i] : i;
                        ent[r].push_back(di);
                        ent[r].push_back(p.raster ? p.r_res[r] : i);
                    }
                continue;
            }
            if (orderS) {
                // A_n(q, R) = sum_k Z_s[t][q][k] C[R][k]
                d.a_off = site_moff[si]; d.lda = p.N1pad; d.a_tstride = (int64_t)p.N2 * p.N1pad;
                d.b_off = 0; d.ldb = p.N1pad;
                d.h_off = -1; d.ldh = 0;
                d.M = p.N2; d.N_inner = Ps; d.n_t = st.n_trans; d.K = p.N1;
                d.idx_off = site_idx[s];
            } else if (p.hs2) {
                // A_n(q, R) = sum_r (H_t S2w)[q][r] Psi_s[i][r]: the producer's H_t S_2w rows
                // (one block per transition), Psi shared by the transitions
                d.a_off = site_m2off[si]; d.lda = p.Kpad; d.a_tstride = (int64_t)p.N2 * p.Kpad;
                d.b_off = site_moff[si]; d.ldb = p.Kpad; d.b_tstride = 0;
                d.h_off = -1; d.ldh = 0;
                d.M = p.N2; d.N_inner = Ps; d.n_t = st.n_trans; d.K = p.K;
                d.idx_off = -1;
            } else {
                // A_n(q, R) = sum_r S2w[q][r] H_t[r] Psi_s[i][r]  (or its band-basis form)
                if (p.recip) { d.a_off = p.slice_w2[pb.slice]; d.lda = p.Kbpad; }
                else { d.a_off = p.slice_w2[pb.slice] + (int64_t)p.site_w2[s] * w2_stride; d.lda = p.Kpad; }
                if (h_in_gemm) {
                    d.b_off = site_moff[si]; d.ldb = p.Kpad;
                    d.h_off = st.h_offset * p.K; d.ldh = p.K;
                } else {
                    d.b_off = site_m2off[si]; d.ldb = Kcpad; d.b_tstride = (int64_t)Ps * Kcpad;
                    d.h_off = -1;
                }
                d.M = p.N2; d.N_inner = Ps; d.n_t = st.n_trans; d.K = Kc;
                d.idx_off = -1;
            }
            d.tiles_m = (int)ceil_div(d.M, rows2);
            d.tiles_n = (int)ceil_div(d.N_inner, GEMM_BN);
            d.tile_start = tiles;
            d.p_off = poff; d.ld_part = (int64_t)d.n_t * d.N_inner;
            poff += (int64_t)d.tiles_m * d.ld_part;
            tiles += d.tiles_m * d.tiles_n * d.n_t;
            int di = (int)p.descs.size();
            p.descs.push_back(d);
            if (p.f > 1)
                for (int i = 0; i < Ps; ++i) {
                    int r = pl ? (*pl)[i] : i;
                    ent[r].push_back(di);
                    ent[r].push_back(i);
                }
        }
        bt.d2_count = (int)p.descs.size() - bt.d2_begin;
        bt.d2_tiles = tiles;
        bt.d2_rows = p.gram ? GEMM_BM : rows2;
        if (p.wgram) {
            // M_s[r][r'] = sum_q conj(S2w[q][r]) S2w[q][r']  (upper 128-tiles, FP32 complex), or in
            // split precision with the G epilogue, G_s = gscale M_s o sum_t conj(H_t) H_t^T in SC
            // (both triangles; the H of the site at h_off, K apart, ld_part transitions)
            bt.dm_begin = (int)p.descs.size();
            // the G epilogue on 128-row tiles, or 256-row ones (tuning key 10 = 1)
            bt.dm_rows = (p.wg_fused && tune_get(TUNE_GRAM_ROWS) != 0) ? 256 : GEMM_BM;
            int tl = 0;
            for (size_t si = 0; si < pb.sites.size(); ++si) {
                const Job& jb = p.jobs[bt.job_begin + si];
                GemmDesc d{};
                d.a_off = jb.s2t_off; d.lda = p.N2p; d.b_off = jb.s2t_off; d.ldb = p.N2p;
                d.h_off = -1; d.idx_off = -1;
                d.p_off = jb.m_off; d.ldc_m = p.Kpad; d.ldc_t = 0;
                if (p.wg_fused) {
                    d.c_off = jb.g_off; d.h_off = jb.h_off; d.ldh = p.K; d.ld_part = jb.nt;
                }
                d.M = p.K; d.N_inner = p.K; d.n_t = 1; d.K = p.N2;
                d.tiles_m = (int)ceil_div(p.K, bt.dm_rows);
                d.tiles_n = (int)ceil_div(p.K, GEMM_BN);
                d.tile_start = tl;
                tl += d.tiles_m * d.tiles_n;
                p.descs.push_back(d);
            }
            bt.dm_count = (int)p.descs.size() - bt.dm_begin;
            bt.dm_tiles = tl;
            // Y_s^T[i][r] = sum_r' Psi_s[i][r'] G_s[r][r']  (complex64 store), or in the raster
            // form Z_s[r][q] = sum_r' G_s[r][r'] S_1w[perm(q)][r'] (the S_1 window's rows gathered
            // into beam-slot order from the window buffer, or in split precision with complex64
            // windows from their SC copy)
            bt.dy_begin = (int)p.descs.size();
            tl = 0;
            for (size_t si = 0; si < pb.sites.size(); ++si) {
                const Job& jb = p.jobs[bt.job_begin + si];
                GemmDesc d{};
                if (p.raster) {
                    d.a_off = jb.g_off; d.lda = p.Kpad;
                    d.b_off = (split && !p.w1_sc) ? jb.s1sc_off : jb.win_off; d.ldb = p.Kpad;
                    d.h_off = -1; d.idx_off = p.r_perm_off;
                    d.c_off = jb.y_off; d.ldc_m = p.N1pad; d.ldc_t = 0;
                    d.M = p.K; d.N_inner = p.N1; d.n_t = 1; d.K = p.K;
                    d.tiles_m = (int)ceil_div(p.K, rows2);
                    d.tiles_n = (int)ceil_div(p.N1, GEMM_BN);
                } else {
                    d.a_off = jb.psi_off; d.lda = p.Kpad; d.b_off = jb.g_off; d.ldb = p.Kpad;
                    d.h_off = -1; d.idx_off = -1;
                    d.c_off = jb.y_off; d.ldc_m = p.Kpad; d.ldc_t = 0;
                    d.M = jb.ps; d.N_inner = p.K; d.n_t = 1; d.K = p.K;
                    d.tiles_m = (int)ceil_div(jb.ps, rows2);
                    d.tiles_n = (int)ceil_div(p.K, GEMM_BN);
                }
                d.tile_start = tl;
                tl += d.tiles_m * d.tiles_n;
                p.descs.push_back(d);
            }
            bt.dy_count = (int)p.descs.size() - bt.dy_begin;
            bt.dy_tiles = tl;
            bt.dy_rows = rows2;
            // every operand of the form stays inside the batch's mid, mid2 and part buffers
            const int64_t k16 = round_up(p.K, 16), n16 = round_up(p.N2, 16);
            for (int k = 0; k < bt.job_count && p.raster; ++k) {
                const Job& jb = p.jobs[bt.job_begin + k];
                const int64_t last_row = (int64_t)(p.K - 1) * p.N1pad + p.N1pad;
                const bool ok = jb.s2t_off + (int64_t)(p.K - 1) * p.N2p + n16 <= m2off &&
                                jb.m_off + (int64_t)(p.K - 1) * p.Kpad + p.K <= m2off &&
                                jb.g_off + (int64_t)(p.K - 1) * p.Kpad + k16 <= m2off &&
                                jb.y_off + last_row <= m2off && jb.xt_off + last_row <= m2off &&
                                (!split || p.w1_sc || jb.s1sc_off + (int64_t)(p.N1 - 1) * p.Kpad + k16 <= m2off) &&
                                jb.part_off + (int64_t)p.r_chunks * p.rM * p.rM <= poff &&
                                n16 <= p.N2p && k16 <= p.Kpad && m2off <= p.mid2_elems && poff <= p.part_elems;
                if (!ok) return fail(EELS_ERR_INTERNAL, "raster-form operands leave their buffers");
            }
            for (int k = 0; k < bt.job_count && !p.raster; ++k) {
                const Job& jb = p.jobs[bt.job_begin + k];
                const int64_t rows_y = std::max(jb.ps, 1) - 1;
                const bool ok = jb.s2t_off + (int64_t)(p.K - 1) * p.N2p + n16 <= m2off &&
                                jb.m_off + (int64_t)(p.K - 1) * p.Kpad + p.K <= m2off &&
                                jb.g_off + (int64_t)(p.K - 1) * p.Kpad + k16 <= m2off &&
                                jb.y_off + rows_y * p.Kpad + k16 <= m2off &&
                                jb.psi_off + rows_y * p.Kpad + k16 <= moff && jb.part_off + jb.ps <= poff &&
                                n16 <= p.N2p && k16 <= p.Kpad && m2off <= p.mid2_elems && moff <= p.mid_elems &&
                                poff <= p.part_elems;
                if (!ok) return fail(EELS_ERR_INTERNAL, "window-Gram operands leave their buffers");
            }
        }
        if (p.wgram) {
            std::vector<int32_t> pj;
            for (int k = 0; k < bt.job_count; ++k) {
                const Job& jb = p.jobs[bt.job_begin + k];
                ProdJob q{jb.w_off, jb.s2t_off, jb.win_off, jb.xt_off, jb.s1sc_off, jb.m_off, jb.g_off, jb.h_off,
                          jb.nt, 0};
                const int32_t* w = (const int32_t*)&q;
                pj.insert(pj.end(), w, w + sizeof(ProdJob) / 4);
            }
            bt.p_jobs = B.append(pj);
        }
        if (p.raster) {
            std::vector<int32_t> rj;
            for (int k = 0; k < bt.job_count; ++k) {
                const Job& jb = p.jobs[bt.job_begin + k];
                const int64_t v[3] = {jb.xt_off, jb.y_off, jb.part_off};
                const int32_t* w = (const int32_t*)v;
                rj.insert(rj.end(), w, w + 6);
            }
            bt.r_jobs = B.append(rj);
        }
        if (p.f > 1 || p.raster) {
            std::vector<int32_t> ptr(p.P + 1, 0), flat;
            for (int r = 0; r < p.P; ++r) {
                flat.insert(flat.end(), ent[r].begin(), ent[r].end());
                ptr[r + 1] = (int32_t)(flat.size() / 2);
            }
            bt.red_ptr = B.append(ptr);
            bt.red_ent = B.append(flat);
            bt.n_entries = (int64_t)flat.size() / 2;
        } else {
            bt.red_ptr = bt.red_ent = -1;   // every site covers every probe in order
            bt.n_entries = 0;
        }
        p.slices[pb.slice].batches.push_back((int)p.batches.size());
        p.batches.push_back(bt);
    }

    // doubles, diagnostics capture table, descriptors
    {
        std::vector<int32_t> t(2 * p.dz.size());
        std::memcpy(t.data(), p.dz.data(), 8 * p.dz.size());
        p.dz_off = B.append(t);
        t.resize(2 * p.probes.size());
        std::memcpy(t.data(), p.probes.data(), 8 * p.probes.size());
        p.probes_off = B.append(t);
        std::vector<int32_t> ptr(p.ny + 1), rec;
        for (int y = 0; y < p.ny; ++y) {
            rec.push_back(0); rec.push_back(y); rec.push_back(0); rec.push_back(p.nx);
            ptr[y + 1] = y + 1;
        }
        ptr[0] = 0;
        p.dbg_ptr = B.append(ptr);
        p.dbg_rec = B.append(rec);
        {
            // EELS detector beams among the band slots, and the aperture beams by live column
            // (conventional multislice)
            std::vector<int32_t> dm(p.Kbpad, 0);
            for (int c = 0; c < p.nlx; ++c) {
                int cs = p.nlx == p.nx ? (c < (p.nx + 1) / 2 ? c : c - p.nx) : (c <= p.hlx ? c : c - p.nlx);
                int h = p.band_h[c];
                for (int r = 0; r <= 2 * h; ++r) {
                    int ks = r <= h ? r : -(2 * h + 1 - r);
                    double kx = cs / p.lx, ky = ks / p.ly;
                    double th = p.lam * std::sqrt(kx * kx + ky * ky);
                    dm[p.band_off[c] + r] = (th >= p.beta_in && th <= p.beta_out) ? 1 : 0;
                }
            }
            p.det_mask_off = B.append(dm);
            std::vector<int32_t> ptr(p.nlx + 1, 0), beams;
            std::vector<std::vector<int32_t>> by_col(p.nlx);
            for (int b = 0; b < p.N1; ++b) by_col[live_col(imod((long long)p.f * p.ab1[2 * b], p.nx))].push_back(b);
            for (int c = 0; c < p.nlx; ++c) {
                beams.insert(beams.end(), by_col[c].begin(), by_col[c].end());
                ptr[c + 1] = (int32_t)beams.size();
            }
            p.col_ptr_off = B.append(ptr);
            p.col_beam_off = B.append(beams.empty() ? std::vector<int32_t>{0} : beams);
            p.n_trans_all = 0;
            std::vector<int32_t> org;
            for (size_t s = 0; s < p.sites.size(); ++s) {
                p.n_trans_all += p.sites[s].n_trans;
                for (int t = 0; t < p.sites[s].n_trans; ++t) {
                    org.push_back(p.sites[s].h_offset + t);
                    org.push_back(imod((long long)p.site_ix0[s] - p.hwx, p.nx));
                    org.push_back(imod((long long)p.site_iy0[s] - p.hwy, p.ny));
                    org.push_back(0);
                }
            }
            p.conv_org_off = B.append(org.empty() ? std::vector<int32_t>{0, 0, 0, 0} : org);
        }
        if (p.n_img > 0) {
            p.img_mask_off = B.append(img_mask);
            // Gram GEMM of the companion images: G[k][k'] = sum_g conj(X[k][g]) X[k'][g] over the
            // ring-masked exit band coefficients X [N_1][Kb pad]
            GemmDesc d{};
            d.a_off = 0; d.lda = p.Kbpad; d.b_off = 0; d.ldb = p.Kbpad;
            d.h_off = -1; d.c_off = 0; d.ldc_m = p.N1pad; d.p_off = 0;
            d.M = p.N1; d.N_inner = p.N1; d.n_t = 1; d.K = p.Kbpad; d.idx_off = -1;
            d.tiles_m = (int)ceil_div(p.N1, GEMM_BM);
            d.tiles_n = (int)ceil_div(p.N1, GEMM_BN);
            d.tile_start = 0;
            p.img_desc = (int)p.descs.size();
            p.descs.push_back(d);
        }
        std::vector<int32_t> dd(p.descs.size() * sizeof(GemmDesc) / 4);
        if (!p.descs.empty()) std::memcpy(dd.data(), p.descs.data(), p.descs.size() * sizeof(GemmDesc));
        p.descs_off = B.append(dd);
    }

    // algorithmic sweep traffic: two passes per beam-slice, each reading and writing the
    // live columns of the beam's plane
    double fwd = 0, rev = 0;
    if (!ion.empty()) {
        if (p.s1_inverse) fwd = (double)(2 * p.nz - ion.front()) * p.N1;   // to the exit and back
        else if (p.s2_retreat) fwd = (double)(ion.back() + 1) * p.N1;     // up to the top site
        else
            for (auto& g : p.groups) fwd += (double)(g.ckpt >= 0 ? g.j_hi - g.j_lo + 1 : g.j_hi + 1) * p.N1;
        rev = p.s2_retreat ? (double)(p.nz + ion.back()) * p.N2           // to the entrance, then back up
                           : (double)(p.nz - ion.front()) * p.N2;
    }
    p.sweep_beam_slices = fwd + rev;
    p.sweep_bytes = p.sweep_beam_slices * 32.0 * p.ny * p.nlx;

    // ---- workspace layout: the S-matrix data first (their offsets do not depend on the
    // probes), then the probe-dependent buffers and the table blob
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += A(bytes); return o; };
    p.off_twx = take(c8 * p.nx);
    p.off_twy = take(c8 * p.ny);
    p.off_T = take(c8 * (size_t)p.nz * p.ny * p.nx);
    p.off_P = take(c8 * (size_t)p.nz * (p.nlx + p.ny));   // separable propagator tables
    p.off_s1 = take(c8 * (size_t)p.N1 * p.ny * p.ldx);
    p.off_s2 = take(c8 * (size_t)p.N2 * p.ny * p.ldx);
    p.off_w1 = take(c8 * (size_t)std::max(p.max_w1, 1) * p.N1 * p.Kpad);
    p.off_w2 = take(c8 * (size_t)std::max<int64_t>(w2_elems, 1));
    p.off_C = take(c8 * (size_t)p.P * p.N1pad);
    p.off_mid = take(c8 * (size_t)std::max<int64_t>(p.mid_elems, 1));
    p.off_mid2 = take(c8 * (size_t)std::max<int64_t>(p.mid2_elems, 1));
    p.off_scratch = take(c8 * (size_t)std::max<int64_t>(p.scratch_elems, 1));
    p.off_part = take(4 * (size_t)std::max<int64_t>(p.part_elems, 1));
    p.off_gtot = take(p.gram ? 16 * (size_t)p.N1 * p.N1 : 16);
    p.off_qpart = take(p.gram ? 8 * (size_t)p.P * ceil_div(p.N1, 64) : 8);
    const bool img = p.n_img > 0;
    p.off_img_exit = take(img ? c8 * (size_t)p.N1 * p.Kbpad : 16);
    p.off_img_masked = take(img ? c8 * (size_t)p.N1 * p.Kbpad : 16);
    p.off_img_part = take(img ? c8 * (size_t)p.N1pad * p.N1pad : 16);
    p.off_img_G = take(img ? 16 * (size_t)p.N1 * p.N1 : 16);
    p.off_img_qpart = take(img ? 8 * (size_t)p.P * ceil_div(p.N1, 64) : 16);
    p.off_img_C = take(img ? c8 * (size_t)p.P * p.N1pad : 16);
    p.off_r_c0 = take(p.raster ? c8 * (size_t)p.N1pad : 16);      // c_k(R_0)
    p.off_r_tw = take(p.raster ? c8 * (size_t)p.rM : 16);          // M-point twiddles
    p.off_ckpt = take(p.n_ckpt > 0 ? (size_t)p.n_ckpt * A(c8 * (size_t)p.N1 * p.ny * p.ldx) : 16);
    p.off_blob = take(p.blob.size() * 4);
    p.ws_bytes = off;
    if (budget > 0 && p.ws_bytes > budget) return fail(EELS_ERR_OOM, "workspace exceeds the memory budget");
    return EELS_OK;
}

static void fnv(uint64_t& h, const void* data, size_t n) {
    const unsigned char* c = (const unsigned char*)data;
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
}

uint64_t s_signature(const Plan& p) {
    uint64_t h = 1469598103934665603ull;
    auto add = [&](const auto& v) { fnv(h, &v, sizeof(v)); };
    add(p.nx); add(p.ny); add(p.lx); add(p.ly); add(p.nz);
    fnv(h, p.dz.data(), p.dz.size() * sizeof(double));
    add(p.lam); add(p.sigma); add(p.alpha); add(p.beta_in); add(p.beta_out); add(p.f); add(p.kmax);
    add(p.full_window); add(p.recip); add(p.resident); add(p.w1_sc); add(p.hwx); add(p.hwy); add(p.Kpad); add(p.Kbpad);
    add(p.w2_sc); add(p.N1); add(p.N2);
    fnv(h, p.ab1.data(), p.ab1.size() * sizeof(int));
    fnv(h, p.ab2.data(), p.ab2.size() * sizeof(int));
    for (size_t s = 0; s < p.sites.size(); ++s) {
        add(p.sites[s].slice); add(p.site_ix0[s]); add(p.site_iy0[s]); add(p.site_w1[s]); add(p.site_w2[s]);
    }
    fnv(h, p.slice_w2.data(), p.slice_w2.size() * sizeof(int64_t));
    add(p.off_T); add(p.off_P); add(p.off_s1); add(p.off_s2); add(p.off_w1); add(p.off_w2);
    return h;
}

// The table blob's size is known only after planning; plan with a reserve, then again
// with the measured size if the budget was missed.
eels_status build_plan(Plan& p, const eels_problem& q) {
    size_t reserve = 64 << 10;
    eels_status s = EELS_OK;
    for (int attempt = 0; attempt < 4; ++attempt) {
        p = Plan{};
        s = build_plan_impl(p, q, reserve);
        if (s != EELS_ERR_OOM || q.max_workspace_bytes == 0) return s;
        size_t need = p.blob.size() * 4 + (64 << 10);
        if (p.blob.empty() || need <= reserve) return s;
        reserve = need;
    }
    return s;
}

}  // namespace eels
