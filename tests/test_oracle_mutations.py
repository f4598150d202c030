"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each test swaps one oracle function for a plausibly wrong variant and checks that
the corresponding pin (conventional == PRISM, translation equivariance, the exact
Schroedinger solution, vanishing H) no longer holds.
"""
import numpy as np
import pytest

import synth
from oracle import conventional, metrics, physics as ph, prism
from oracle.common import make_setup

import test_oracle_pins as pins


def _o1_o2_gap(p):
    return metrics.rel_l2(prism.prism_map(p), conventional.conventional_map(p))


def _problem():
    return synth.random_problem(31, n=32, L=8.0, nz=4, n_sites=2, n_trans=2)


def test_printed_transpose_order_equals_exact_for_annular_detector(monkeypatch):
    """The operator order printed in Eq. MSTop (F T F^-1 P) yields S_2 rows of the
    parity-mirrored beam -q.  For an annular (centrosymmetric) detector the set of rows
    is the same, so the map is unchanged; the exact transpose is kept anyway."""
    def reverse_printed(prob, st, j_stop=0):
        N2 = st.ab2.shape[0]
        x = np.zeros((N2, prob.ny, prob.nx), dtype=complex)
        x[np.arange(N2), st.iy2, st.ix2] = 1.0
        for j in range(prob.n_slices - 1, j_stop - 1, -1):
            S2 = st.T[j] * np.fft.ifft2(st.P[j] * x) * (prob.nx * prob.ny)
            yield j, S2
            x = np.fft.fft2(S2) / (prob.nx * prob.ny)
    p = _problem()
    exact = prism.prism_map(p)
    monkeypatch.setattr(prism, "reverse_s2", reverse_printed)
    assert metrics.rel_l2(prism.prism_map(p), exact) < 1e-12


def test_forward_instead_of_transposed_operator_is_caught(monkeypatch):
    def reverse_forward(prob, st, j_stop=0):
        N2 = st.ab2.shape[0]
        x = np.zeros((N2, prob.ny, prob.nx), dtype=complex)
        x[np.arange(N2), st.iy2, st.ix2] = 1.0
        for j in range(prob.n_slices - 1, j_stop - 1, -1):
            S2 = np.fft.ifft2(x) * (prob.nx * prob.ny)
            yield j, S2
            x = st.P[j] * np.fft.fft2(st.T[j] * np.fft.ifft2(x))
    monkeypatch.setattr(prism, "reverse_s2", reverse_forward)
    assert _o1_o2_gap(_problem()) > 1e-8   # the pin holds to 1e-12


def test_dropped_transmission_of_ionising_slice_is_caught(monkeypatch):
    """S_2(j) without the slice's own transmission factor (the inelastic wave skipping
    T_j) breaks conventional == PRISM."""
    orig = prism.contract_site

    def contract_without_Tj(prob, st, s, S1j, S2j, I):
        orig(prob, st, s, S1j, S2j / st.T[int(prob.site_slice[s])][None], I)
    monkeypatch.setattr(prism, "contract_site", contract_without_Tj)
    assert _o1_o2_gap(_problem()) > 1e-8


def test_probe_phase_sign_is_caught(monkeypatch):
    orig = ph.probe_coefficients

    def flipped(*a, **k):
        return np.conj(orig(*a, **k))
    monkeypatch.setattr(ph, "probe_coefficients", flipped)
    p = synth.random_problem(8, n=32, L=8.0, nz=3, n_sites=2)
    sx, sy = 5, 3
    dx, dy = p.lx / p.nx, p.ly / p.ny
    q = p.replace(V=np.roll(p.V, (sy, sx), axis=(1, 2)), H=np.roll(p.H, (sy, sx), axis=(1, 2)),
                  site_xy=p.site_xy + [sx * dx, sy * dy], probes=p.probes + [sx * dx, sy * dy])
    assert not np.allclose(prism.prism_map(q), prism.prism_map(p), rtol=1e-6)


def test_propagator_sign_is_caught(monkeypatch):
    orig = ph.propagator

    def flipped(*a, **k):
        return np.conj(orig(*a, **k))
    monkeypatch.setattr(ph, "propagator", flipped)
    with pytest.raises(AssertionError):
        pins.test_split_step_converges_to_exact_schroedinger_solution()


def test_transmission_sign_is_caught(monkeypatch):
    orig = ph.transmission
    monkeypatch.setattr(ph, "transmission", lambda V, s: np.conj(orig(V, s)))
    with pytest.raises(AssertionError):
        pins.test_split_step_converges_to_exact_schroedinger_solution()


def test_dropped_transition_potential_is_caught(monkeypatch):
    import oracle.prism as pr
    monkeypatch.setattr(pr, "site_H", lambda prob, s, n: np.ones(prob.H.shape[1:], dtype=complex))
    with pytest.raises(AssertionError):
        pins.test_zero_transition_gives_zero()


# --- interpolation f > 1: the tiled-specimen identity bites ----------------------------

def test_dropped_f2_detector_weight_is_caught(monkeypatch):
    orig = prism.contract_windows
    monkeypatch.setattr(prism, "contract_windows", lambda S1w, S2w, C, Hs, f2: orig(S1w, S2w, C, Hs, 1.0))
    assert pins.tiled_identity_gaps(2)[0] > 1e-3


def test_wrong_probe_scale_for_interpolation_is_caught(monkeypatch):
    """s = f / sqrt(N_1(f = 1)) instead of f^2 / sqrt(N_1(f = 1))."""
    orig = ph.probe_coefficients

    def scaled(ab, lx, ly, f, *a, **k):
        c = orig(ab, lx, ly, f, *a, **k)
        return c / f if f > 1 else c
    monkeypatch.setattr(ph, "probe_coefficients", scaled)
    assert pins.tiled_identity_gaps(2)[0] > 1e-3


def test_wrong_eligibility_box_is_caught(monkeypatch):
    """The crop box compared with an L/(2f) box instead of the L/f box."""
    orig = ph.eligible

    def halved(ix0, iy0, hx, hy, nx, ny, lx, ly, f, probes):
        return orig(ix0, iy0, hx, hy, nx, ny, lx, ly, 2 * f if f > 1 else f, probes)
    monkeypatch.setattr(ph, "eligible", halved)
    assert pins.tiled_identity_gaps(2)[0] > 1e-3


@pytest.mark.parametrize("wrong", ["quarter", "lambda_cubed", "sign"])
def test_wrong_spherical_aberration_term_is_caught(monkeypatch, wrong):
    """A C_s term with a quarter instead of a half, one more power of lambda, or the opposite
    sign moves the aberrated probe's centroid off the transverse ray aberration."""
    import math

    def chi_wrong(k2, lam, defocus_A=0.0, cs_A=0.0):
        c = {"quarter": 0.25 * cs_A * lam * lam, "lambda_cubed": 0.5 * cs_A * lam ** 3,
             "sign": -0.5 * cs_A * lam * lam}[wrong]
        return math.pi * lam * k2 * (c * k2 - defocus_A)
    monkeypatch.setattr(ph, "aberration_chi", chi_wrong)
    with pytest.raises(AssertionError):
        pins.test_spherical_aberration_transverse_ray_aberration(5e5, 0.0)
