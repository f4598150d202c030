"""GPU frozen-phonon averaging against the oracle's average over the same configurations."""
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
    from paper_1908_07628_amd import eels, phonon
    return eels, phonon


def _configs(u, n=3):
    return [synth.random_problem(41, n=64, L=10.0, nz=4, n_sites=3, n_trans=2, aperture_mrad=18.0,
                                 det_outer_mrad=28.0, displace_A=u, displace_seed=100 + i) for i in range(n)]


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_frozen_phonon_mean_matches_oracle(prec, tol):
    eels, phonon = _gpu()
    cfg = _configs(0.1)
    mean, per = phonon.frozen_phonon_map(cfg, precision=prec)
    ref = prism.frozen_phonon_map(cfg)
    assert maps_close(mean, ref, tol)
    assert per.shape == (3, cfg[0].n_probes)
    assert np.std(per, axis=0).max() > 0              # the configurations differ


def test_zero_displacement_gives_the_static_map():
    eels, phonon = _gpu()
    cfg = _configs(0.0)
    mean, per = phonon.frozen_phonon_map(cfg, precision="fp32")
    static = eels.solve(cfg[0])
    assert np.array_equal(per[0], static) and np.array_equal(per[2], static)
