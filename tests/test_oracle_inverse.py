"""Pins of the inverse multislice (oracle/prism.py: inverse_s1 and inverse_s2, Sec. 4.C)."""
import numpy as np

import synth
from oracle import metrics, prism
from oracle.common import make_setup


def _cell(seed=21, nz=4, **kw):
    base = dict(n=64, L=10.0, nz=nz, n_sites=3, n_trans=2, aperture_mrad=18.0, det_outer_mrad=28.0)
    base.update(kw)
    return synth.random_problem(seed, **base)


def test_free_space_inverse_is_exact():
    """V = 0: T = 1 and |P| = 1 on the band, so retreating undoes propagation exactly."""
    p = _cell()
    p = p.replace(V=np.zeros_like(p.V))
    st = make_setup(p)
    js = list(range(p.n_slices))
    a, b = prism.forward_s1(p, st, js), prism.inverse_s1(p, st, js)
    for j in js:
        assert np.allclose(a[j], b[j], rtol=0, atol=1e-13)


def test_uniform_potential_inverse_is_exact():
    """A constant potential is a pure phase: nothing leaves the band, M^-1 M = 1 exactly."""
    p = _cell(seed=22)
    p = p.replace(V=np.full_like(p.V, 37.5))
    st = make_setup(p)
    js = list(range(p.n_slices))
    a, b = prism.forward_s1(p, st, js), prism.inverse_s1(p, st, js)
    for j in js:
        assert np.allclose(a[j], b[j], rtol=0, atol=1e-12)
    assert metrics.rel_l2(prism.prism_map(p, s1_mode="inverse"), prism.prism_map(p)) < 1e-12


def test_inverse_error_grows_with_scattering_strength():
    """With scattering beyond the band the inverse loses what the band limit removed: the map
    error is nonzero, small, and grows with the potential's strength (more intensity is
    pushed past the band limit)."""
    errs = []
    for k in (1.0, 4.0, 16.0):
        p = _cell(seed=23, nz=6, atoms_per_slice=6, widths=(0.15, 0.5), amp=(30.0 * k, 8.0 * k))
        errs.append(metrics.rel_l2(prism.prism_map(p, s1_mode="inverse"), prism.prism_map(p)))
    assert 1e-9 < errs[0] < errs[1] < errs[2] < 0.01


def _s2_exact(p, st, js):
    return {j: S2 for j, S2 in prism.reverse_s2(p, st, j_stop=0) if j in set(js)}


def test_free_space_s2_retreat_is_exact():
    """V = 0: retreating S_2 from the entrance undoes each transposed step exactly."""
    p = _cell(seed=24)
    p = p.replace(V=np.zeros_like(p.V))
    st = make_setup(p)
    js = list(range(p.n_slices))
    a, b = _s2_exact(p, st, js), prism.inverse_s2(p, st, js)
    for j in js:
        assert np.allclose(a[j], b[j], rtol=0, atol=1e-12)


def test_uniform_potential_s2_retreat_is_exact():
    """A constant potential is a pure phase: the retreated S_2 equals the transposed sweep's at
    every slice, and the map equals the exact one."""
    p = _cell(seed=25)
    p = p.replace(V=np.full_like(p.V, 21.0))
    st = make_setup(p)
    js = list(range(p.n_slices))
    a, b = _s2_exact(p, st, js), prism.inverse_s2(p, st, js)
    for j in js:
        assert np.allclose(a[j], b[j], rtol=0, atol=1e-12)
    assert metrics.rel_l2(prism.prism_map(p, s1_mode="inverse_s2"), prism.prism_map(p)) < 1e-12


def test_s2_retreat_entrance_slice_is_exact_and_error_grows_with_strength():
    """S_2 at the entrance comes from the exact sweep, so a specimen ionised only in slice 0
    gives the exact map whatever the potential; with sites higher up the error is nonzero,
    small, and grows with the potential's strength."""
    p = _cell(seed=26, nz=5, atoms_per_slice=6, widths=(0.15, 0.5), amp=(240.0, 64.0))
    keep = np.nonzero(p.site_slice == 0)[0]
    if keep.size == 0:
        keep = np.array([0])
        p = p.replace(site_slice=np.zeros_like(p.site_slice))
    p0 = p.replace(site_slice=p.site_slice[keep], site_xy=p.site_xy[keep], site_ntrans=p.site_ntrans[keep],
                   site_hoff=p.site_hoff[keep])
    assert metrics.rel_l2(prism.prism_map(p0, s1_mode="inverse_s2"), prism.prism_map(p0)) < 1e-12
    errs = []
    for k in (1.0, 4.0, 16.0):
        q = _cell(seed=23, nz=6, atoms_per_slice=6, widths=(0.15, 0.5), amp=(30.0 * k, 8.0 * k))
        errs.append(metrics.rel_l2(prism.prism_map(q, s1_mode="inverse_s2"), prism.prism_map(q)))
    assert 1e-9 < errs[0] < errs[1] < errs[2] < 0.01
