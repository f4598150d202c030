"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each pin checks the oracle against something other than itself: a printed number,
a closed form, an independent algorithm (conventional vs PRISM, exact ODE solution
vs split-step), an invariant, or brute force on a tiny input.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg

import synth
from synth.specimens import Problem
from oracle import conventional, metrics, models, physics as ph, prism
from oracle.common import make_setup

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed.json")))
LAM300 = ph.wavelength_A(300e3)


# --------------------------------------------------------------------------- constants

def test_wavelength_and_sigma_closed_forms():
    # independent textbook forms: lambda = 12.2643 / sqrt(V (1 + 0.978476e-6 V)) A and
    # sigma = 2 pi / (lambda V) * (m0 c^2 + e V) / (2 m0 c^2 + e V)
    for V in (80e3, 200e3, 300e3):
        lam_k = 12.26426 / math.sqrt(V * (1.0 + 0.9784756e-6 * V))
        assert ph.wavelength_A(V) == pytest.approx(lam_k, rel=2e-6)
        mc2 = 510998.95
        sig_k = 2 * math.pi / (ph.wavelength_A(V) * V) * (mc2 + V) / (2 * mc2 + V)
        assert ph.sigma_per_VA(V) == pytest.approx(sig_k, rel=1e-9)
    assert ph.wavelength_A(300e3) == pytest.approx(GOLD["wavelength_300keV"]["lambda_A"], abs=1e-6)
    assert ph.sigma_per_VA(300e3) == pytest.approx(6.53e-4, rel=1e-3)


# --------------------------------------------------------------------------- printed numbers

def test_memory_example_printed():
    g = GOLD["memory_example"]
    ms, tr, sm = models.memory_bytes(g["N"], g["n_z"], g["N1"], g["N2"])
    assert g["half_side"] == g["N"] // 2
    # the paper truncates: 107.9 MB, 1.214 GB, 4.382 GB
    assert math.floor(ms / 1e6) == g["ms_minimum_MB"]
    assert math.floor(tr / 1e7) / 100 == g["transmission_GB"]
    assert math.floor(sm / 1e7) / 100 == g["smatrices_GB"]


def test_beam_count_printed():
    g = GOLD["beam_count_example"]
    f = 9
    L = g["L_over_f_A"] * f
    ab, _, _ = ph.lattice_beams(1836, 1836, L, L, f, LAM300, 0.0, g["alpha_mrad"] * 1e-3)
    assert ab.shape[0] == g["N1"]
    # and the count agrees with the pi alpha^2 L^2 / f^2 estimate of Sec. 3
    assert models.beam_count_estimate(g["alpha_mrad"] * 1e-3, LAM300, L, f) == pytest.approx(325, rel=0.01)


def test_nyquist_step_printed():
    g = GOLD["nyquist_step"]
    assert round(models.nyquist_probe_step(g["alpha_mrad"] * 1e-3, LAM300), 3) == g["step_A"]


def test_config_beam_counts():
    # aperture / detector beam counts of the synthetic workloads (inclusive edges)
    def count(n, L, f, lo, hi):
        return ph.lattice_beams(n, n, L, L, f, LAM300, lo * 1e-3, hi * 1e-3)[0].shape[0]
    assert count(64, 10.0, 1, 0, 20) == 325
    assert count(64, 10.0, 1, 0, 40) == 1305
    assert count(256, 20.0, 1, 0, 21) == 1433
    assert count(256, 20.0, 1, 0, 50) == 8093
    assert count(1024, 100.0, 4, 0, 20) == 2025
    assert count(1024, 100.0, 4, 0, 40) == 8093


def test_op_counts():
    # the sum form equals n_states n_z (n_z+1)/2 + n_z (brute force), which differs from
    # the printed closed form n_states n_z (n_z-1)/2 + n_z by n_states n_z.
    for ns in (1, 3, 9):
        for nz in (1, 2, 5, 50):
            brute = 0
            for iz in range(nz):
                for _ in range(ns):
                    brute += nz - iz
            brute += nz
            assert models.ms_ops_sum(ns, nz) == brute
            assert models.ms_ops_sum(ns, nz) - models.ms_ops_printed(ns, nz) == ns * nz


# --------------------------------------------------------------------------- error metric

def test_error_metric_known_values():
    # Eq. nrmsse read as ||a - b||_2 / ||b||_2, worked by hand: a - b = (3, -4) has norm 5
    # and ||b|| = 4, so 1.25 (a dropped square root would give 25/16)
    assert metrics.rel_l2([3.0, 0.0], [0.0, 4.0]) == pytest.approx(1.25, abs=1e-15)
    # (1, 2, 2) against (1, 0, 0): sqrt(0 + 4 + 4) / 1
    assert metrics.rel_l2([1.0, 2.0, 2.0], [1.0, 0.0, 0.0]) == pytest.approx(math.sqrt(8.0), abs=1e-15)
    # equal maps, and a zero reference (then the norm of a itself)
    assert metrics.rel_l2([2.0, -1.0], [2.0, -1.0]) == 0.0
    assert metrics.rel_l2([3.0, 4.0], [0.0, 0.0]) == pytest.approx(5.0, abs=1e-15)
    # max pointwise error over the largest reference value: max |(-1, 1)| / max |(2, 4)|
    assert metrics.max_rel([1.0, 5.0], [2.0, 4.0]) == pytest.approx(0.25, abs=1e-15)
    # signs: |(-3) - 1| = 4 over max |(1, -8)| = 8
    assert metrics.max_rel([-3.0, -8.0], [1.0, -8.0]) == pytest.approx(0.5, abs=1e-15)
    # scale invariance of both (a relative metric)
    rng = np.random.default_rng(3)
    a, b = rng.standard_normal(50), rng.standard_normal(50)
    assert metrics.rel_l2(7 * a, 7 * b) == pytest.approx(metrics.rel_l2(a, b), rel=1e-14)
    assert metrics.max_rel(7 * a, 7 * b) == pytest.approx(metrics.max_rel(a, b), rel=1e-14)


# --------------------------------------------------------------------------- aberrations

@pytest.mark.parametrize("cs_A,defocus_A", [(5e5, 0.0), (-5e5, 0.0), (5e5, 60.0)])
def test_spherical_aberration_transverse_ray_aberration(cs_A, defocus_A):
    # Geometric optics fixes the C_s term of Eq. illum independently of how chi is written:
    # a ray leaving the probe-forming lens at angle theta lands theta (C_s theta^2 - defocus)
    # from the axis (third-order transverse aberration), and by the Fourier shift theorem a
    # narrow bundle of plane waves with phases -chi(k) forms a packet centred at grad chi / 2 pi.
    # So the intensity centroid of a probe built from a small off-axis aperture must sit at the
    # bundle's mean of theta_x (C_s theta^2 - defocus), here several angstrom away from 0.
    n, L, lam = 256, 40.0, LAM300
    k0, dk = 0.025 / lam, 0.25                     # 25 mrad off axis, 0.25 1/A bundle radius
    a = np.arange(-n // 2, n // 2)
    AX, AY = np.meshgrid(a, a, indexing="xy")
    KX, KY = AX / L, AY / L
    inside = (KX - k0) ** 2 + KY ** 2 <= dk * dk
    k2 = KX ** 2 + KY ** 2
    chi = ph.aberration_chi(k2, lam, defocus_A=defocus_A, cs_A=cs_A)
    spec = np.zeros((n, n), dtype=np.complex128)
    spec[np.mod(AY[inside], n), np.mod(AX[inside], n)] = np.exp(-1j * chi[inside])
    psi = np.fft.ifft2(spec)
    ix = np.abs(psi) ** 2
    prof_x, prof_y = ix.sum(axis=0), ix.sum(axis=1)
    x = np.arange(n) * L / n
    cx = L / (2 * np.pi) * np.angle(np.sum(prof_x * np.exp(2j * np.pi * x / L)))   # circular mean
    cy = L / (2 * np.pi) * np.angle(np.sum(prof_y * np.exp(2j * np.pi * x / L)))
    th_x, th2 = lam * KX[inside], lam * lam * k2[inside]
    expect = float(np.mean(th_x * (cs_A * th2 - defocus_A)))
    assert abs(expect) > 3.0                          # a displacement the test can see
    assert cx == pytest.approx(expect, rel=0.03)
    assert abs(cy) < 0.02 * abs(expect)               # the bundle is symmetric in y


# --------------------------------------------------------------------------- transforms

def test_fft_convention_brute_force():
    # forward transform carries exp(-2 pi i r.g) (footnote to Eq. 4)
    rng = np.random.default_rng(0)
    n = 6
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    r = np.arange(n)
    W = np.exp(-2j * np.pi * np.outer(r, r) / n)
    brute = W @ x @ W
    assert np.allclose(np.fft.fft2(x), brute, atol=1e-12)
    assert np.allclose(np.fft.ifft2(brute), x, atol=1e-12)


# --------------------------------------------------------------------------- propagation

def _free_problem(n=32, L=8.0, nz=3, aperture=20.0, **kw):
    p = synth.random_problem(5, n=n, L=L, nz=nz, aperture_mrad=aperture, **kw)
    return p.replace(V=np.zeros_like(p.V))


def test_free_space_plane_wave_is_pure_phase():
    p = _free_problem()
    st = make_setup(p)
    S1 = prism.forward_s1(p, st, [p.n_slices - 1])[p.n_slices - 1]
    z = float(np.sum(p.dz[:-1]))
    for b in range(st.ab1.shape[0]):
        kx = st.ab1[b, 0] / p.lx
        ky = st.ab1[b, 1] / p.ly
        X, Y = np.meshgrid(np.arange(p.nx) * p.lx / p.nx, np.arange(p.ny) * p.ly / p.ny)
        expect = np.exp(-1j * np.pi * st.lam * z * (kx * kx + ky * ky)) * \
            np.exp(2j * np.pi * (kx * X + ky * Y)) / (p.nx * p.ny)
        assert np.allclose(S1[b], expect, atol=1e-14)


def test_band_limit_removes_beams_outside():
    p = _free_problem(n=16, L=4.0, nz=2)
    st = make_setup(p)
    kmax = ph.band_radius(16, 16, 4.0, 4.0)
    KX, KY = ph.kgrid(16, 16, 4.0, 4.0)
    outside = np.sqrt(KX ** 2 + KY ** 2) > kmax
    assert np.all(st.P[0][outside] == 0)
    assert np.all(np.abs(st.P[0][~outside]) == pytest.approx(1.0))


def test_norm_preserved_without_potential_and_not_increased_with_it():
    rng = np.random.default_rng(1)
    p = synth.random_problem(7, n=32, L=8.0, nz=6)
    st = make_setup(p)
    mask = ph.band_mask(32, 32, 8.0, 8.0) > 0
    x = (rng.standard_normal((32, 32)) + 1j * rng.standard_normal((32, 32))) * mask
    n0 = np.linalg.norm(x)
    y = x.copy()
    for j in range(p.n_slices):  # V = 0
        y = st.P[j] * np.fft.fft2(np.fft.ifft2(y))
    assert np.linalg.norm(y) == pytest.approx(n0, rel=1e-13)
    y, prev = x.copy(), n0
    for j in range(p.n_slices):  # V != 0
        y = st.P[j] * np.fft.fft2(st.T[j] * np.fft.ifft2(y))
        nn = np.linalg.norm(y)
        assert nn <= prev * (1 + 1e-13)
        prev = nn
    assert prev < n0  # the band limit does remove the scattered tail


def _ode_problem(nslices, z_total=40.0):
    n, L = 8, 4.0
    X, Y = np.meshgrid(np.arange(n) * L / n, np.arange(n) * L / n)
    V3 = 5.0 + 15.0 * np.cos(2 * np.pi * X / L) + 10.0 * np.sin(2 * np.pi * (X + 2 * Y) / L)
    dz = z_total / nslices
    p = synth.random_problem(1, n=n, L=L, nz=nslices, n_sites=0, dz=[dz] * nslices,
                             aperture_mrad=0.6 * LAM300 * 1e3, det_outer_mrad=12.0)
    return p.replace(V=np.repeat((V3 * dz)[None].astype(np.float32), nslices, axis=0)), V3


def test_split_step_converges_to_exact_schroedinger_solution():
    """Eq. Spsi solved exactly by a matrix exponential of the coupled equations Eq. Schro
    (restricted to the band-limited components) vs the multislice of Eq. 4 / Eq. MSop."""
    errs = []
    for ns in (5, 10, 20, 40):
        p, V3 = _ode_problem(ns)
        st = make_setup(p)
        n = p.nx
        mask = (ph.band_mask(n, n, p.lx, p.ly) > 0).ravel()
        KX, KY = ph.kgrid(n, n, p.lx, p.ly)
        k2 = (KX ** 2 + KY ** 2).ravel()
        # reciprocal-space potential operator: x_hat -> fft2(V3 * ifft2(x_hat))
        # (V3 is float32-rounded through the problem; use the same values)
        V3r = p.V[0].astype(np.float64) / p.dz[0]
        Vop = np.zeros((n * n, n * n), dtype=complex)
        for c in range(n * n):
            e = np.zeros(n * n, dtype=complex)
            e[c] = 1
            Vop[:, c] = np.fft.fft2(V3r * np.fft.ifft2(e.reshape(n, n))).ravel()
        G = -1j * np.pi * st.lam * np.diag(k2) + 1j * st.sigma * Vop
        Pm = np.diag(mask.astype(float))
        U = scipy.linalg.expm(Pm @ G @ Pm * float(np.sum(p.dz)))
        S = prism.forward_s1(p, st, [ns - 1])[ns - 1]  # entrance of the last slice
        err = 0.0
        for b in range(st.ab1.shape[0]):
            x_last = np.fft.fft2(S[b])
            x_exit = st.P[ns - 1] * np.fft.fft2(st.T[ns - 1] * np.fft.ifft2(x_last))
            col = np.ravel_multi_index((st.iy1[b], st.ix1[b]), (n, n))
            err = max(err, np.max(np.abs(x_exit.ravel() - U[:, col])))
        errs.append(err)
    assert errs[-1] < 2e-3
    for a, b in zip(errs, errs[1:]):
        assert b < 0.6 * a  # first-order (or better) convergence in the slice thickness


def test_defocus_moves_with_propagation():
    """A probe with defocus df, propagated through dz of vacuum, is the probe with defocus
    df - dz (the aberration phase of Eq. illum and the Fresnel factor of Eq. MSop agree)."""
    df, dz = 30.0, 12.0
    p = _free_problem(n=32, L=10.0, nz=1).replace(dz=np.array([dz]), defocus_A=df,
                                                   probes=np.array([[3.0, 4.0]]), probe_shape=(1, 1))
    st = make_setup(p)
    x = np.zeros((32, 32), dtype=complex)
    x[st.iy1, st.ix1] = st.C[:, 0]
    y = st.P[0] * np.fft.fft2(st.T[0] * np.fft.ifft2(x))
    q = p.replace(defocus_A=df - dz)
    st2 = make_setup(q)
    z = np.zeros((32, 32), dtype=complex)
    z[st2.iy1, st2.ix1] = st2.C[:, 0]
    assert np.allclose(y, z, atol=1e-14)


# --------------------------------------------------------------------------- transpose

def test_exact_transpose_identity():
    """sum_r S_2(j)[q](r) phi(r) equals the forward multislice of phi from slice j to the
    exit, evaluated at detector beam q, for random phi."""
    rng = np.random.default_rng(3)
    p = synth.random_problem(11, n=24, ny=20, L=7.0, Ly=6.0, nz=4, det_inner_mrad=5.0,
                             det_outer_mrad=21.0)
    st = make_setup(p)
    for j, S2 in prism.reverse_s2(p, st, 0):
        phi = rng.standard_normal((p.ny, p.nx)) + 1j * rng.standard_normal((p.ny, p.nx))
        x = phi
        for jj in range(j, p.n_slices):
            x = st.P[jj] * np.fft.fft2(st.T[jj] * (x if jj == j else np.fft.ifft2(x)))
        lhs = np.einsum("qyx,yx->q", S2, phi)
        assert np.allclose(lhs, x[st.iy2, st.ix2], rtol=1e-12, atol=1e-12)


# --------------------------------------------------------------------------- contraction

def test_zero_transition_gives_zero():
    p = synth.config1()
    p0 = p.replace(H=np.zeros_like(p.H))
    assert np.all(prism.prism_map(p0) == 0)
    assert np.all(conventional.conventional_map(p0) == 0)


def test_intensity_quadratic_in_H():
    p = synth.random_problem(2, n=32, L=8.0, nz=3)
    a = 0.7 - 1.3j
    I1 = prism.prism_map(p)
    I2 = prism.prism_map(p.replace(H=(a * p.H.astype(np.complex128)).astype(np.complex128)))
    assert np.allclose(I2, abs(a) ** 2 * I1, rtol=1e-12)


def test_additive_over_sites():
    p = synth.random_problem(3, n=32, L=8.0, nz=4, n_sites=3)
    total = prism.prism_map(p)
    parts = prism.site_maps(p)
    assert np.allclose(parts.sum(axis=0), total, rtol=1e-12)
    # each part is the map of that site alone
    for s in range(p.n_sites):
        sel = np.array([s])
        ps = p.replace(site_slice=p.site_slice[sel], site_xy=p.site_xy[sel],
                       site_ntrans=p.site_ntrans[sel], site_hoff=p.site_hoff[sel])
        assert np.allclose(prism.prism_map(ps), parts[s], rtol=1e-12)


def test_vacuum_closed_form():
    """V = 0: I(R) = sum_{q in D} |B(q) fft2(H psi_j)(q)|^2 with psi_j the free-space probe
    at the slice of the transition (no multislice needed)."""
    p = synth.random_problem(4, n=32, L=8.0, nz=4, n_sites=1, n_trans=2, det_inner_mrad=3.0,
                             det_outer_mrad=25.0)
    p = p.replace(V=np.zeros_like(p.V))
    st = make_setup(p)
    j = int(p.site_slice[0])
    z = float(np.sum(p.dz[:j]))
    KX, KY = ph.kgrid(p.nx, p.ny, p.lx, p.ly)
    k2 = KX ** 2 + KY ** 2
    B = np.sqrt(k2) <= ph.band_radius(p.nx, p.ny, p.lx, p.ly)
    th = st.lam * np.sqrt(k2)
    D = (th >= 3e-3) & (th <= 25e-3)
    expect = np.zeros(p.n_probes)
    for R in range(p.n_probes):
        c = np.zeros((p.ny, p.nx), dtype=complex)
        c[st.iy1, st.ix1] = st.C[:, R]
        psi = np.fft.ifft2(np.exp(-1j * np.pi * st.lam * z * k2) * c)
        for n in range(2):
            expect[R] += np.sum(np.abs(B * np.fft.fft2(p.H[n] * psi))[D] ** 2)
    assert np.allclose(prism.prism_map(p), expect, rtol=1e-11)
    assert np.allclose(conventional.conventional_map(p), expect, rtol=1e-11)


def test_unit_transition_in_vacuum_gives_unit_intensity():
    p = synth.random_problem(6, n=32, L=8.0, nz=3, n_sites=1, n_trans=1, det_outer_mrad=25.0)
    p = p.replace(V=np.zeros_like(p.V), H=np.ones_like(p.H))
    assert np.allclose(prism.prism_map(p), 1.0, rtol=1e-12)


# --------------------------------------------------------------------------- whole method

@pytest.mark.parametrize("kw", [
    dict(seed=21, n=16, L=5.0, nz=2),
    dict(seed=22, n=32, L=8.0, nz=4, n_sites=3, n_trans=3),
    dict(seed=23, n=32, ny=24, L=9.0, Ly=7.0, nz=3, det_inner_mrad=8.0, det_outer_mrad=22.0),
    dict(seed=24, n=48, L=10.0, nz=3, window_A=3.0, n_sites=2),
    dict(seed=25, n=32, L=8.0, nz=3, defocus_A=40.0, cs_A=1e7),
    dict(seed=26, n=64, L=12.0, nz=2, dz=[1.5, 2.5], n_sites=2, window_A=5.0),
])
def test_conventional_equals_prism(kw):
    """O1 (conventional multislice) and O2 (PRISM with the exact transpose) compute the
    same map (Sec. 4.A compares them; in FP64 they agree to rounding)."""
    kw = dict(kw)
    p = synth.random_problem(kw.pop("seed"), **kw)
    I1 = conventional.conventional_map(p)
    I2 = prism.prism_map(p)
    assert np.max(I1) > 0
    assert metrics.rel_l2(I2, I1) < 1e-12


def test_config1_conventional_equals_prism():
    p = synth.config1()
    assert metrics.rel_l2(prism.prism_map(p), conventional.conventional_map(p)) < 1e-12


def test_translation_equivariance():
    p = synth.random_problem(8, n=32, L=8.0, nz=3, n_sites=2)
    sx, sy = 5, 3
    dx, dy = p.lx / p.nx, p.ly / p.ny
    q = p.replace(V=np.roll(p.V, (sy, sx), axis=(1, 2)),
                  H=np.roll(p.H, (sy, sx), axis=(1, 2)),
                  site_xy=p.site_xy + [sx * dx, sy * dy],
                  probes=p.probes + [sx * dx, sy * dy])
    assert np.allclose(prism.prism_map(q), prism.prism_map(p), rtol=1e-10)


def test_crop_converges_to_full_cell():
    """Cropping the contraction (Sec. 4.B): the error against the full-cell map falls as the
    window grows, and is tiny once the window holds the transition potential."""
    base = synth.random_problem(9, n=64, L=12.0, nz=3, n_sites=1, n_trans=2)
    full = prism.prism_map(base)
    errs = []
    for W in (1.0, 2.0, 3.0, 5.0, 8.0):
        pc = synth.random_problem(9, n=64, L=12.0, nz=3, n_sites=1, n_trans=2, window_A=W)
        errs.append(metrics.rel_l2(prism.prism_map(pc), full))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-4


def test_interpolation_window_invariant():
    """f > 1, V = 0, H = 1 on a window that holds the probe: the detected intensity is
    close to 1 (what the probe carries inside its L/f box)."""
    p = synth.random_problem(10, n=128, L=24.0, nz=2, n_sites=1, n_trans=1, window_A=9.0,
                             interp_f=2, aperture_mrad=25.0, det_outer_mrad=34.0,
                             probes=[[12.0, 12.0], [11.0, 12.5]])
    p = p.replace(V=np.zeros_like(p.V), H=np.ones_like(p.H),
                  site_xy=np.array([[12.0, 12.0]]))
    I = prism.prism_map(p)
    assert np.all(I > 0.95) and np.all(I < 1.0 + 1e-9)


def test_interpolation_factor_one_matches_fine_lattice_reference():
    # f = 1 with a crop equals the conventional map with H zero outside the window
    p = synth.random_problem(12, n=48, L=10.0, nz=3, window_A=4.0, n_sites=2, interp_f=1)
    assert metrics.rel_l2(prism.prism_map(p), conventional.conventional_map(p)) < 1e-12


@pytest.mark.parametrize("kw", [
    dict(seed=31, n=32, L=8.0, nz=4, n_sites=3, n_trans=3),
    dict(seed=32, n=48, ny=32, L=10.0, Ly=7.0, nz=3, window_A=3.0, n_sites=2, det_inner_mrad=6.0,
         det_outer_mrad=24.0),
])
def test_beam_split_map_equals_conventional(kw):
    """The map regrouped by beams (disjoint aperture and detector beam sets, uneven parts)
    equals the conventional multislice map (the plain definition) to rounding."""
    kw = dict(kw)
    p = synth.random_problem(kw.pop("seed"), **kw)
    I1 = conventional.conventional_map(p)
    for parts, chunk in ((1, 1000), (3, 5), (7, 2)):
        assert metrics.rel_l2(prism.prism_map_by_beams(p, n_parts=parts, chunk=chunk), I1) < 1e-12


def test_beam_split_map_with_interpolation_and_crop():
    """f = 2 with cropped windows (the nanoparticle form): the beam-split map equals the
    stored-S map, and probes that see no site get exactly zero."""
    p = synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=4, f=2)
    far = np.array([[1.0, 1.0]])          # a probe whose L/f box holds no crop box
    p = p.replace(probes=np.concatenate([p.probes, far]), probe_shape=(1, p.n_probes + 1))
    ref = prism.prism_map(p)
    got = prism.prism_map_by_beams(p, n_parts=4, chunk=7)
    assert np.max(ref) > 0
    assert metrics.rel_l2(got, ref) < 1e-12
    st = make_setup(p)
    from oracle.common import site_eligible
    seen = np.any([site_eligible(p, st, s) for s in range(p.n_sites)], axis=0)
    assert not seen[-1] and seen.sum() >= 1
    assert np.all(got[~seen] == 0.0) and np.all(got[seen] > 0)


def test_mirror_maps_m_to_minus_m():
    """A cell mirror-symmetric under y -> L - y (no jitter; atoms asymmetric in x) with the
    ionised atom on the mirror line: the map of transition m at probe R equals the map of
    -m at the mirrored probe, since the mirror takes the azimuth phi to -phi.  The maps of m
    and -m themselves differ, so the pin checks the sign of the azimuth through the whole
    method."""
    from synth.specimens import _finish, ENERGY_300KEV, probe_grid
    L, n, nz, ns = 10.0, 48, 3, 6
    xs = (1.0, 4.0, 7.5)
    a_slice, a_xy = [], []
    for j in range(nz):
        for x in xs:
            for iy in range(3):
                a_slice.append(j)
                a_xy.append((x, (iy + 0.5) * L / 3))
    amp = np.tile([[40.0, 10.0]], (len(a_slice), 1))
    wid = np.tile([[0.3, 0.8]], (len(a_slice), 1))
    probes = probe_grid(ns, ns, L / ns, L / ns)
    maps = {}
    for m in (-1, 1, -2, 2):
        p = _finish("mirror", n, n, L, L, [2.0] * nz, a_slice, a_xy, amp, wid, [1], [(4.0, L / 2)],
                    [(abs(m), m, 0.4)], probes, (ns, ns), energy_eV=ENERGY_300KEV, aperture_mrad=20.0,
                    det_inner_mrad=0.0, det_outer_mrad=30.0, interp_f=1, window_A=0.0)
        maps[m] = prism.prism_map(p)
    iy, ix = np.divmod(np.arange(ns * ns), ns)
    mirror = ((ns - iy) % ns) * ns + ix
    for m in (1, 2):
        top = np.max(maps[m])
        assert np.max(np.abs(maps[m] - maps[-m][mirror])) < 1e-9 * top
        assert np.max(np.abs(maps[m] - maps[-m])) > 1e-5 * top      # 4 orders above rounding


def test_window_not_smaller_than_cell_is_the_full_cell():
    """A crop window at least as large as the cell means the full cell: the map equals the
    uncropped map exactly."""
    full = synth.random_problem(13, n=32, L=8.0, nz=3, n_sites=2, n_trans=2, window_A=0.0)
    big = synth.random_problem(13, n=32, L=8.0, nz=3, n_sites=2, n_trans=2, window_A=8.0)
    assert big.H.shape == full.H.shape
    assert np.array_equal(prism.prism_map(big), prism.prism_map(full))


def tiled_identity_gaps(f, ny=32, Ly=8.0, aberr=None):
    """The tiled-specimen identity for f > 1 (see the test below): returns the largest
    deviation of the f > 1 map from f^2 N_1 / N_1(f = 1) times the small cell's
    conventional map at probes that see a copy (relative to that map's maximum), the
    largest f > 1 value at probes that see none, the factor, and the small cell's smallest
    value there relative to its maximum."""
    ps = synth.random_problem(41, n=32, ny=ny, L=8.0, Ly=Ly, nz=3, n_sites=1, n_trans=3, window_A=4.0,
                              aperture_mrad=15.0, det_outer_mrad=20.0, **(aberr or {}))
    copies = np.array([ps.site_xy[0] + [i * ps.lx, j * ps.ly] for j in range(f) for i in range(f)])
    rng = np.random.default_rng(5)
    # the crop box (2 A half-width) lies inside the probe's L/f box for |dx| <= 2 A, |dy| <= Ly/2 - 2 A
    near = np.concatenate([c + rng.uniform(-1, 1, (3, 2)) * [1.5, 0.8] for c in copies])
    far = copies + [ps.lx / 2, ps.ly / 2]            # half a small cell from every copy
    pb = synth.tiled_problem(ps, f, np.concatenate([near, far]))
    big = prism.prism_map(pb)
    small = conventional.conventional_map(ps.replace(probes=np.mod(pb.probes, [ps.lx, ps.ly]),
                                                     probe_shape=(1, pb.n_probes)))
    st = make_setup(pb)
    ratio = f * f * st.ab1.shape[0] / st.n1_fine
    n = len(near)
    return (float(np.max(np.abs(big[:n] - ratio * small[:n])) / np.max(small[:n])),
            float(np.max(np.abs(big[n:]))), ratio, float(np.min(small[n:]) / np.max(small)))


@pytest.mark.parametrize("f,ny,Ly,aberr", [(2, 32, 8.0, {}), (3, 24, 6.0, {}), (4, 32, 8.0, {}),
                                           (2, 32, 8.0, dict(defocus_A=40.0, cs_A=2.0e6))])
def test_interpolation_on_a_tiled_specimen_equals_the_small_cell(f, ny, Ly, aberr):
    """A specimen made of f x f copies of a small cell (every ionised site copied too): the
    coarse PRISM lattice of the big cell is the full lattice of the small cell and every
    S-matrix row repeats with the small cell's period, so for a probe R that sees a copy the
    f > 1 map equals the conventional multislice map of the small cell at R mod (L/f), times
    f^2 N_1 / N_1(f = 1) (the f^2 detector weight and the probe scale s_f against the small
    cell's unit-norm probe).  A probe whose L/f box holds no crop box gets exactly zero.
    The identity also holds with defocus and spherical aberration (the same phase at the
    same beams)."""
    near_gap, far_max, ratio, far_small = tiled_identity_gaps(f, ny, Ly, aberr)
    assert abs(ratio - 1.0) > 1e-3                  # the factor is visible at this aperture
    assert near_gap <= 1e-12
    assert far_max == 0.0 and far_small > 1e-6
