"""Full-size parity at the benchmark workloads, in the launch configurations bench.py times,
against FP64 values of the oracle at sampled probes:

* the whole nanoparticle map (config 3: 1024^2, 50 slices, 22,659 sites x 9 transitions,
  f = 4, 4 A crop, order P, window-Gram detector sum, memory budget from the free HBM) at
  64 probes over the central 32 x 32 of the raster (tests/golden/config3_map_samples.json,
  written by make_config3_map_samples.py), BF16 split and FP32;
* the crystal map (config 2: 650 sites x 9 transitions, 4096 probes; band basis, order S,
  Gram detector sum) at 16 probes, dark ones included, of the conventional-multislice oracle
  (tests/golden/config2_samples.json, written by make_config2_samples.py), BF16 split and FP32;
* the sites of the nanoparticle's most populated slice (config3_samples.json) with both
  detector sums and all precisions.

Each case bounds the relative L2 error (Eq. nrmsse reading) and every sample's error against
the largest sampled value, and the relative error of every sample that carries at least a
hundredth of that value."""
import json
import os
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden", "config2_samples.json")


def _bounds(got, ref, bar, per_sample):
    err = np.abs(got - ref)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < bar          # Eq. nrmsse reading
    assert np.max(err) <= bar * np.max(ref)                                  # every sample
    lit = ref >= 1e-2 * np.max(ref)
    assert np.all(err[lit] <= per_sample * ref[lit])                         # each lit sample


@pytest.mark.parametrize("precision,bar", [("bf16_split", 1e-3), ("fp32", 1e-4)])
def test_config2_sampled_probes(precision, bar):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    g = json.load(open(GOLD))
    p = synth.config2()
    print(f"config2 generated; solving {precision}", flush=True)
    sys.stdout.flush()
    m = eels.solve(p, precision=precision)
    ref = np.asarray(g["map"])
    got = m[g["probe_index"]]
    print("sampled", got, "ref", ref, flush=True)
    assert len(ref) >= 16 and np.min(ref) < 0.05 * np.max(ref)             # dark probes are sampled
    assert np.all(np.isfinite(m)) and np.all(m >= 0)
    _bounds(got, ref, bar, 5 * bar)


GOLD3M = os.path.join(os.path.dirname(__file__), "golden", "config3_map_samples.json")


@pytest.mark.parametrize("precision,bar", [("bf16_split", 1e-3), ("fp32", 1e-4)])
def test_config3_whole_map_sampled_probes(precision, bar):
    """The whole nanoparticle map as bench.py computes it (all 40 ionised slices, the slice
    groups and site batches its memory budget gives, window-Gram detector sum), at the 64
    stored probes."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD3M):
        pytest.skip("config3_map_samples.json not written (tests/golden/make_config3_map_samples.py)")
    from paper_1908_07628_amd import eels
    g = json.load(open(GOLD3M))
    p = synth.config3()
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    print(f"config3 generated ({p.n_sites} sites); solving the whole map in {precision}", flush=True)
    plan = eels.Plan(p, precision=precision, max_workspace_bytes=int(free - (8 << 30) - (4 << 30)))
    info = plan.info()
    assert info["window_gram_form"] == 1 and info["n_ion_slices"] == len(set(p.site_slice.tolist()))
    V, H = eels.device_inputs(p)
    ws = plan.alloc_workspace()
    out = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    plan.execute(V, H, out, ws)
    torch.cuda.synchronize()
    m = out.cpu().numpy()
    del ws, V, H, out
    torch.cuda.empty_cache()
    ref = np.asarray(g["map"])
    got = m[g["probe_index"]]
    print("groups", info["n_groups"], "batches", info["n_batches"], "sampled", got[:6], "ref", ref[:6], flush=True)
    assert np.all(np.isfinite(m)) and np.all(m >= 0)
    assert np.all(ref > 0) and len(ref) == 64
    _bounds(got, ref, bar, 2 * bar)


GOLD3 = os.path.join(os.path.dirname(__file__), "golden", "config3_samples.json")


@pytest.mark.parametrize("precision,bar,wgram", [("bf16_split", 1e-3, 0), ("fp16_split", 1e-3, 0), ("fp32", 1e-4, 0),
                                                 ("bf16_split", 1e-3, 1), ("fp16_split", 1e-3, 1), ("fp32", 1e-4, 1)])
def test_config3_sampled_probes(precision, bar, wgram):
    """Full-size nanoparticle geometry (1024^2, 50 slices, f = 4, 4 A crop, N_1 = N_2 = 2025)
    in the launch configuration of bench.py's nanoparticle workload (order P, memory budget
    from the free HBM), on the 1217 sites of the most populated ionised slice; sampled
    probes against the FP64 PRISM oracle (tests/golden/config3_samples.json, written by
    make_config3_samples.py), with the per-transition and the window-Gram detector sums.
    Probes whose L/f box holds no crop box are exactly zero."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLD3):
        pytest.skip("config3_samples.json not written (tests/golden/make_config3_samples.py)")
    from paper_1908_07628_amd import eels
    g = json.load(open(GOLD3))
    p = synth.config3()
    sel = np.nonzero(p.site_slice == g["slice"])[0]
    assert len(sel) == g["n_sites"]
    q = p.replace(site_slice=p.site_slice[sel], site_xy=p.site_xy[sel], site_ntrans=p.site_ntrans[sel],
                  site_hoff=p.site_hoff[sel])
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    print(f"config3 slice {g['slice']} ({len(sel)} sites) generated; solving {precision}", flush=True)
    keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, wgram)     # detector sum: per transition or window Gram
        m = eels.solve(q, precision=precision, max_workspace_bytes=int(free - (8 << 30) - (4 << 30)))
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
    torch.cuda.empty_cache()
    ref = np.asarray(g["map"])
    got = m[g["probe_index"]]
    print("sampled", got[:8], "ref", ref[:8], flush=True)
    assert np.all(np.isfinite(m)) and np.all(m >= 0)
    assert np.all(got[ref == 0.0] == 0.0)
    lit = ref > 0
    assert lit.sum() >= 32
    _bounds(got, ref, bar, 5 * bar)
