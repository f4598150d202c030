"""Pins of the inverse-multislice S_1 (oracle/prism.py: inverse_s1, Sec. 4.C)."""
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
