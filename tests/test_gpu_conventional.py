"""GPU conventional multislice EELS (Sec. 3, first algorithm) through the C ABI, against the
FP64 conventional-multislice oracle on small cells, against the FP64 samples of the
full config-2 workload, and against the GPU scattering-matrix map (which equals it at
interpolation factor 1).  FP32 waves: map rel-L2 <= 1e-4."""
import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle import conventional, metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config2_samples.json")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    return eels


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_conv(eels, p, chunk):
    plan = eels.Plan(p)
    V, H = eels.device_inputs(p)
    ws = torch.empty(plan.conventional_workspace_bytes(chunk), dtype=torch.uint8, device="cuda")
    out = torch.full((plan.n_probes,), -1.0, dtype=torch.float64, device="cuda")
    plan.conventional_map(V, H, out, chunk, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _cases():
    c = {}
    c["config1"] = synth.config1()
    c["rand_square"] = synth.random_problem(3, n=32, nz=4, n_sites=3, n_trans=2)
    # sites in the first and (two of them) the last slice, a rectangular cell
    q = synth.random_problem(5, n=32, ny=64, L=8.0, Ly=16.0, nz=5, n_sites=3, n_trans=3)
    c["rand_rect_last_slice"] = q.replace(site_slice=np.array([0, 4, 4], dtype=q.site_slice.dtype))
    # windowed transition potentials (scattered into full planes), annular detector,
    # aberrated probe
    c["rand_window_annular"] = synth.random_problem(7, n=64, L=12.0, nz=3, n_sites=2, n_trans=2, window_A=5.0,
                                                    det_inner_mrad=8.0, det_outer_mrad=30.0, defocus_A=40.0,
                                                    cs_A=1e4)
    return c


@pytest.mark.parametrize("name", ["config1", "rand_square", "rand_rect_last_slice", "rand_window_annular"])
def test_conventional_against_oracle(name):
    eels = _need_gpu()
    p = _cases()[name]
    _say("conventional", name, p.nx, p.ny, p.n_slices, p.n_sites, p.n_probes)
    ref = conventional.conventional_map(p)
    # a chunk that leaves a ragged last chunk, and all probes at once
    for chunk in (max(1, p.n_probes // 2 - 1), p.n_probes):
        got = _gpu_conv(eels, p, chunk)
        err = metrics.rel_l2(got, ref)
        _say(" chunk", chunk, "rel-L2", err)
        assert err < 1e-4, (chunk, err)


def test_conventional_chunks_bitwise():
    """Every wave is computed on its own, so the map does not depend on the probe chunk."""
    eels = _need_gpu()
    p = _cases()["rand_square"]
    _say("conventional chunks", p.n_probes)
    a = _gpu_conv(eels, p, 1)
    b = _gpu_conv(eels, p, 4)
    c = _gpu_conv(eels, p, p.n_probes)
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_conventional_no_transitions_zero():
    """H = 0 gives a zero map (the zero-transition pin of the oracle, on the GPU)."""
    eels = _need_gpu()
    p = synth.random_problem(11, n=32, nz=3, n_sites=2, n_trans=2)
    p = p.replace(H=np.zeros_like(p.H))
    _say("conventional H=0")
    got = _gpu_conv(eels, p, p.n_probes)
    assert np.all(got == 0.0)


def test_conventional_config2_sampled_probes():
    """The full config-2 specimen (650 sites x 9 transitions, 50 slices) at the probes whose
    FP64 conventional map values are stored."""
    eels = _need_gpu()
    g = json.load(open(GOLD))
    p = synth.config2()
    idx = np.asarray(g["probe_index"])
    q = p.replace(probes=p.probes[idx], probe_shape=(1, len(idx)))
    _say("conventional config2 samples", len(idx))
    got = _gpu_conv(eels, q, len(idx))
    ref = np.asarray(g["map"])
    _say(" got", got, "ref", ref)
    err = np.abs(got - ref)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-4      # Eq. nrmsse reading
    assert np.max(err) <= 1e-4 * np.max(ref)                            # every sample
    lit = ref >= 1e-2 * np.max(ref)
    assert np.all(err[lit] <= 1e-3 * ref[lit])                          # each lit sample


def test_conventional_matches_prism_config2_subset():
    """At f = 1 the scattering-matrix contraction is the conventional map: the two GPU
    paths agree on a 4 x 4 block of the config-2 raster."""
    eels = _need_gpu()
    p = synth.config2()
    idx = np.array([iy * 64 + ix for iy in range(20, 24) for ix in range(30, 34)])
    q = p.replace(probes=p.probes[idx], probe_shape=(4, 4))
    _say("conventional vs prism config2", len(idx))
    conv = _gpu_conv(eels, q, 8)
    prism = eels.solve(q, precision="fp32")
    err = metrics.rel_l2(conv, prism)
    _say(" rel-L2", err)
    assert err < 1e-4
