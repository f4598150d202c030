"""Write config3_samples.json: FP64 PRISM map values (f = 4, 4 A crop) of the full-size
nanoparticle workload (synth.config3: 1024 x 1024 px, 50 slices, N_1 = N_2 = 2025) at
sampled probe positions, for the sites of the ionised slice with the most sites; computed
with the PRISM oracle only (oracle.prism.prism_map_by_beams, the beams split over worker
processes).

Cost: every aperture and detector beam is multisliced on its own through about 51 slices
of 1024 x 1024 (about 2e5 plane FFTs): roughly an hour on 8 cores.

Usage: python tests/golden/make_config3_samples.py [n_workers]
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import prism  # noqa: E402

# an 8 x 8 lattice of raster positions (step 32 px = 12.5 A), offset from the atom lattice;
# the corners lie outside the particle, where no site is eligible
PROBES_IX_IY = [(19 + 32 * a, 23 + 32 * b) for b in range(8) for a in range(8)]
N_SCAN = 256


def sample_problem():
    """The slice subset and sampled probes the stored values belong to."""
    p = synth.config3()
    counts = np.bincount(p.site_slice, minlength=p.n_slices)
    j = int(np.argmax(counts))
    sel = np.nonzero(p.site_slice == j)[0]
    return p, j, sel


def main():
    nw = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    p, j, sel = sample_problem()
    idx = np.array([iy * N_SCAN + ix for ix, iy in PROBES_IX_IY])
    rows = np.concatenate([np.arange(p.site_hoff[s], p.site_hoff[s] + p.site_ntrans[s]) for s in sel])
    hoff = np.concatenate([[0], np.cumsum(p.site_ntrans[sel])[:-1]]).astype(p.site_hoff.dtype)
    q = p.replace(site_slice=p.site_slice[sel], site_xy=p.site_xy[sel], site_ntrans=p.site_ntrans[sel],
                  site_hoff=hoff, H=p.H[rows], probes=p.probes[idx], probe_shape=(8, 8))
    print(f"slice {j}: {len(sel)} sites; {len(idx)} probes; setup {time.time() - t0:.0f} s", flush=True)
    with mp.get_context("fork").Pool(nw) as pool:
        I = prism.prism_map_by_beams(q, n_parts=nw, chunk=8, map_fn=pool.imap)
    out = {
        "about": "FP64 PRISM EELS map (f = 4, 4 A crop) of the full-size nanoparticle workload "
                 "(synth.config3) restricted to the sites of its most populated ionised slice, at "
                 "sampled probes; written by tests/golden/make_config3_samples.py (oracle only)",
        "slice": j,
        "n_sites": int(len(sel)),
        "probes_ix_iy": PROBES_IX_IY,
        "probe_index": [int(v) for v in idx],
        "map": [float(v) for v in I],
        "seconds": round(time.time() - t0, 1),
        "workers": nw,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_samples.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
