"""GPU parity of the inverse-multislice S_1 (Sec. 4.C) against the oracle's inverse mode,
and its size of error against the exact (stored-window) path."""
import sys

import numpy as np
import pytest

from maptol import maps_close
import synth
from oracle import metrics, prism

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    return eels


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "config1": lambda: synth.config1(),
    "strong_full_cell": lambda: synth.random_problem(31, n=64, L=10.0, nz=6, n_sites=4, n_trans=2,
                                                     atoms_per_slice=6, widths=(0.15, 0.5), amp=(120.0, 32.0),
                                                     aperture_mrad=18.0, det_outer_mrad=28.0),
    "crop_window": lambda: synth.random_problem(32, n=128, L=16.0, nz=5, n_sites=4, n_trans=2, window_A=3.0,
                                                aperture_mrad=20.0, det_outer_mrad=30.0, n_scan=4),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("order", ["s_first", "probe_first"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_inverse_multislice_matches_oracle(name, order, prec, tol):
    eels = _gpu()
    p = CASES[name]()
    _say("inverse", name, order, prec)
    ref = prism.prism_map(p, s1_mode="inverse")
    g = eels.solve(p, precision=prec, order=order, s1_mode="inverse")
    assert maps_close(g, ref, tol)


def test_inverse_multislice_error_against_exact_path():
    """The approximation's size on the GPU equals the oracle's: both compare the inverse and
    stored paths of the same map."""
    eels = _gpu()
    p = CASES["strong_full_cell"]()
    exact_o = prism.prism_map(p)
    inv_o = prism.prism_map(p, s1_mode="inverse")
    e_oracle = metrics.rel_l2(inv_o, exact_o)
    g_exact = eels.solve(p)
    g_inv = eels.solve(p, s1_mode="inverse")
    e_gpu = metrics.rel_l2(g_inv, g_exact)
    _say("inverse error oracle", e_oracle, "gpu", e_gpu)
    assert 1e-7 < e_oracle < 0.01
    assert abs(e_gpu - e_oracle) < 0.1 * e_oracle + 2e-5


def test_inverse_multislice_exact_for_uniform_potential_and_images_unchanged():
    eels = _gpu()
    p = synth.random_problem(33, n=128, L=12.0, nz=4, n_sites=3, n_trans=2, aperture_mrad=20.0,
                             det_outer_mrad=30.0, n_scan=4, widths=(0.12, 0.4))
    u = p.replace(V=np.full_like(p.V, 25.0))
    assert metrics.rel_l2(eels.solve(u, s1_mode="inverse"), eels.solve(u)) < 1e-5
    rings = [(0.0, 30.0), (60.0, 0.0)]
    m1, i1 = eels.solve_with_images(p, rings)
    m2, i2 = eels.solve_with_images(p, rings, s1_mode="inverse")
    assert np.array_equal(i1, i2)          # same forward sweep to the exit


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("order", ["s_first", "probe_first"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_s2_retreat_matches_oracle(name, order, prec, tol):
    """S_2 formed at the entrance and retreated towards the exit (Sec. 4.C as printed)."""
    eels = _gpu()
    p = CASES[name]()
    _say("inverse_s2", name, order, prec)
    ref = prism.prism_map(p, s1_mode="inverse_s2")
    g = eels.solve(p, precision=prec, order=order, s1_mode="inverse_s2")
    assert maps_close(g, ref, tol)


def test_s2_retreat_error_against_exact_path():
    eels = _gpu()
    p = CASES["strong_full_cell"]()
    exact_o = prism.prism_map(p)
    inv_o = prism.prism_map(p, s1_mode="inverse_s2")
    e_oracle = metrics.rel_l2(inv_o, exact_o)
    g_exact = eels.solve(p)
    g_inv = eels.solve(p, s1_mode="inverse_s2")
    e_gpu = metrics.rel_l2(g_inv, g_exact)
    _say("inverse_s2 error oracle", e_oracle, "gpu", e_gpu)
    assert 1e-7 < e_oracle < 0.05
    assert abs(e_gpu - e_oracle) < 0.1 * e_oracle + 2e-5


def test_s2_retreat_exact_for_uniform_potential_and_images_unchanged():
    eels = _gpu()
    p = synth.random_problem(34, n=128, L=12.0, nz=4, n_sites=3, n_trans=2, aperture_mrad=20.0,
                             det_outer_mrad=30.0, n_scan=4, widths=(0.12, 0.4))
    u = p.replace(V=np.full_like(p.V, 25.0))
    assert metrics.rel_l2(eels.solve(u, s1_mode="inverse_s2"), eels.solve(u)) < 1e-5
    rings = [(0.0, 30.0), (60.0, 0.0)]
    m1, i1 = eels.solve_with_images(p, rings)
    m2, i2 = eels.solve_with_images(p, rings, s1_mode="inverse_s2")
    assert np.array_equal(i1, i2)          # same forward sweep to the exit


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16_split", 1e-3)])
def test_s2_retreat_entrance_slice_is_exact(prec, tol):
    """At slice 0 the retreat takes the transposed sweep's own capture, so a one-slice specimen
    (and the entrance slice of any) gives the stored path's map."""
    eels = _gpu()
    p = synth.random_problem(35, n=64, L=10.0, nz=1, n_sites=3, n_trans=2, atoms_per_slice=6,
                             widths=(0.15, 0.5), amp=(120.0, 32.0), aperture_mrad=18.0, det_outer_mrad=28.0)
    ref = prism.prism_map(p, s1_mode="inverse_s2")
    assert metrics.rel_l2(ref, prism.prism_map(p)) < 1e-12
    assert maps_close(eels.solve(p, precision=prec, s1_mode="inverse_s2"), ref, tol)


@pytest.mark.parametrize("wgram", [0, 2])
def test_s2_retreat_interpolated_crop_cell(wgram):
    """The S_2 retreat with interpolation factor 2 and 4 A crop windows (the nanoparticle's
    geometry on a small cell), with the per-transition products and with the window-Gram
    detector sum, in BF16 split, against the oracle's inverse_s2 map."""
    eels = _gpu()
    p = synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2)
    ref = prism.prism_map(p, s1_mode="inverse_s2")
    keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, wgram)
        _say("inverse_s2 f=2 crop, window-Gram key", wgram)
        g = eels.solve(p, precision="bf16_split", order="probe_first", s1_mode="inverse_s2")
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
    assert maps_close(g, ref, 1e-3)
    assert np.all(g[ref == 0] == 0)


@pytest.mark.parametrize("mode", ["inverse", "inverse_s2"])
@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_inverse_modes_in_the_raster_form(mode, prec):
    """Both inverse multislice modes with the raster form forced (its S_1 windows captured SC
    with c_k(R_0) folded in, by the inverse row pass for the S_1 retreat and by the forward
    row pass beside the S_2 retreat), against the oracle's map of the same mode."""
    eels = _gpu()
    p = synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2)
    ref = prism.prism_map(p, s1_mode=mode)
    keep = (eels.tune_get(eels.TUNE_WINDOW_GRAM), eels.tune_get(eels.TUNE_RASTER))
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
        eels.tune_set(eels.TUNE_RASTER, 2)
        assert eels.Plan(p, precision=prec, order="probe_first", s1_mode=mode).info()["raster_form"] == 64
        _say("raster form", mode, prec)
        g = eels.solve(p, precision=prec, order="probe_first", s1_mode=mode)
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep[0])
        eels.tune_set(eels.TUNE_RASTER, keep[1])
    assert maps_close(g, ref, 1e-3)
    assert np.all(g[ref == 0] == 0)
