"""Pins of the companion-image oracle (oracle/images.py) against what the physics fixes."""
import numpy as np
import pytest

import synth
from oracle import images, physics as ph
from oracle.common import make_setup


def _cell(seed=5, **kw):
    base = dict(n=64, L=9.0, nz=3, n_sites=1, n_trans=1, aperture_mrad=20.0, det_outer_mrad=30.0)
    base.update(kw)
    return synth.random_problem(seed, **base)


def test_free_space_images_are_the_aperture_fraction_inside_the_ring():
    """V = 0: T = 1, so |psi_hat(g)|^2 = |c_g|^2 = 1/N_1 on the aperture pixels for every probe;
    a ring collects (aperture beams inside it) / N_1, independent of the probe position."""
    p = _cell()
    p = p.replace(V=np.zeros_like(p.V))
    st = make_setup(p)
    lam = st.lam
    kk = lam * np.sqrt((st.ab1[:, 0] / p.lx) ** 2 + (st.ab1[:, 1] / p.ly) ** 2)
    n1 = len(kk)
    for (a, b) in [(0.0, 10.0), (5.0, 15.0), (0.0, 30.0), (12.0, None)]:
        inside = (kk >= a * 1e-3) & ((kk <= b * 1e-3) if b else True)
        got = images.detector_images(p, [(a, b)])[0]
        assert np.allclose(got, inside.sum() / n1, rtol=1e-12, atol=1e-14)


def test_ring_additivity_and_beam_conservation():
    """Disjoint rings add up; with V = 0 the whole band holds the full beam, and with a
    potential the band holds at most the beam (the band limit only removes intensity)."""
    p = _cell(seed=7)
    lam = ph.wavelength_A(p.energy_eV)
    split = 14.123   # mrad, between lattice radii
    total = images.detector_images(p, [(0.0, None)])[0]
    parts = images.detector_images(p, [(0.0, split), (split + 1e-9, None)])
    assert np.allclose(parts.sum(axis=0), total, rtol=1e-12)
    assert np.all(total <= 1.0 + 1e-12) and np.all(total > 0.5)
    free = images.detector_images(p.replace(V=np.zeros_like(p.V)), [(0.0, None)])[0]
    assert np.allclose(free, 1.0, rtol=1e-12)


def test_exit_wave_matches_single_probe_conventional_route():
    """The batched exit waves equal the conventional oracle's one-probe routine."""
    from oracle import conventional
    p = _cell(seed=9)
    psi = images.exit_waves(p, [0, 3])
    assert np.allclose(psi[0], conventional.elastic_exit(p, 0), rtol=1e-12, atol=1e-15)
    assert np.allclose(psi[1], conventional.elastic_exit(p, 3), rtol=1e-12, atol=1e-15)


def test_bf_corrected_is_the_ratio():
    assert np.allclose(images.bf_corrected([2.0, 3.0], [4.0, 6.0]), [0.5, 0.5])


def test_images_refuse_interpolation_factor():
    p = synth.config3_subproblem(n=128, L=25.0, nz=2, n_scan=2, f=2)
    with pytest.raises(ValueError):
        images.detector_images(p, [(0.0, 10.0)])
