"""Write config4_samples.json: FP64 PRISM map values of three specimens of the 64-specimen
batch workload (synth.config4: the cheapest 128^2 specimen, f = 1, the cheapest 256^2 one,
f = 2, and the cheapest 384^2 one, f = 3, all with 4 A crop windows) at sampled probe
positions, computed with the PRISM oracle only (oracle.prism.prism_map on the sampled probes).

Usage: python tests/golden/make_config4_samples.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import prism  # noqa: E402

N_SAMPLES = 16


def picks(specs):
    """Index of the cheapest specimen (grid x slices) of each of the grids 128, 256 and 384."""
    out = []
    for n in (128, 256, 384):
        cand = [i for i, p in enumerate(specs) if p.nx == n]
        out.append(min(cand, key=lambda i: (specs[i].n_slices, i)))
    return out


def sample_index(p):
    """N_SAMPLES probes spread over the raster (seeded)."""
    rng = np.random.default_rng(4)
    return np.sort(rng.choice(p.n_probes, size=min(N_SAMPLES, p.n_probes), replace=False))


def main():
    t0 = time.time()
    specs = synth.config4(n_specimens=64, workers=min(8, os.cpu_count() or 1))
    out = {"about": "FP64 PRISM EELS maps of three specimens of the batch workload (synth.config4, 64 "
                    "specimens) at sampled probes; written by tests/golden/make_config4_samples.py "
                    "(oracle only)",
           "specimens": []}
    for i in picks(specs):
        p = specs[i]
        idx = sample_index(p)
        q = p.replace(probes=p.probes[idx], probe_shape=(1, len(idx)))
        t1 = time.time()
        m = prism.prism_map(q)
        print(f"specimen {i}: {p.nx}^2, {p.n_slices} slices, {p.n_sites} sites, f = {p.interp_f}: "
              f"{time.time() - t1:.0f} s", flush=True)
        out["specimens"].append({"index": int(i), "nx": int(p.nx), "n_slices": int(p.n_slices),
                                 "interp_f": int(p.interp_f), "probe_index": [int(v) for v in idx],
                                 "map": [float(v) for v in m]})
    out["seconds"] = round(time.time() - t0, 1)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_samples.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out)[:400])


if __name__ == "__main__":
    main()
