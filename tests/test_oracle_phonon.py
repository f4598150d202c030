"""Pins of the frozen-phonon inputs and average (synth.thermal_displacement, oracle)."""
import numpy as np

import synth
from oracle import prism


def test_displacement_statistics_and_identity():
    xy = np.random.default_rng(0).uniform(0, 30.0, size=(20000, 2))
    same = synth.thermal_displacement(xy, 30.0, 30.0, 0.0, 3)
    assert np.array_equal(same, xy)
    d = synth.thermal_displacement(xy, 30.0, 30.0, 0.1, 3) - xy
    d = (d + 15.0) % 30.0 - 15.0                       # undo the periodic wrap
    assert abs(d.mean()) < 0.003 and abs(d.std() - 0.1) < 0.003
    a = synth.thermal_displacement(xy, 30.0, 30.0, 0.1, 3)
    b = synth.thermal_displacement(xy, 30.0, 30.0, 0.1, 4)
    assert np.array_equal(a, synth.thermal_displacement(xy, 30.0, 30.0, 0.1, 3)) and not np.array_equal(a, b)


def test_sites_move_with_their_atoms():
    p0 = synth.random_problem(5, n=64, L=10.0, nz=3, n_sites=2)
    p1 = synth.random_problem(5, n=64, L=10.0, nz=3, n_sites=2, displace_A=0.1, displace_seed=1)
    assert 0 < np.abs(p1.site_xy - p0.site_xy).max() < 1.0
    # the transition potential of site 0 is the same function re-centred: its peak moves with it
    h0 = np.abs(p0.H[0]); h1 = np.abs(p1.H[0])
    assert np.isclose(h0.sum(), h1.sum(), rtol=1e-3)


def test_frozen_phonon_average_of_identical_configurations_is_the_static_map():
    p = synth.config1()
    assert np.allclose(prism.frozen_phonon_map([p, p, p]), prism.prism_map(p), rtol=1e-14)
