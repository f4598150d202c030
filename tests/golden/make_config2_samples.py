"""Write config2_samples.json: FP64 map values of the full config-2 workload at a few
probe positions, computed with the conventional multislice oracle only.

The conventional map is a sum over sites of independent contributions (the elastic
wave does not depend on the sites), so sites are split over worker processes.

Usage: python tests/golden/make_config2_samples.py [n_workers]
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
from oracle import conventional  # noqa: E402

# (ix, iy) on the 64 x 64 raster (0.3125 A steps, 4 A lattice period = 12.8 steps): next to a
# B column, on an A column, between columns, near another B column; then A-column and
# O-column positions far from every ionised B column (the darkest parts of the map), points
# on the lines between columns, and a spread over the rest of the cell
PROBES_IX_IY = [(6, 6), (0, 0), (19, 13), (45, 57),
                (13, 13), (26, 0), (0, 39), (51, 51),
                (6, 0), (0, 6), (32, 19), (19, 32),
                (3, 10), (29, 44), (58, 22), (40, 3)]
_P = None


def _work(site_idx):
    """The map contribution of a subset of the sites at the sampled probes."""
    p = _P
    sel = np.asarray(site_idx, dtype=np.int64)
    idx = np.array([iy * 64 + ix for ix, iy in PROBES_IX_IY])
    q = p.replace(site_slice=p.site_slice[sel], site_xy=p.site_xy[sel], site_ntrans=p.site_ntrans[sel],
                  site_hoff=p.site_hoff[sel], probes=p.probes[idx], probe_shape=(1, len(idx)))
    return conventional.conventional_map(q, probe_chunk=len(idx))


def main():
    global _P
    nw = int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count()
    t0 = time.time()
    _P = synth.config2()
    chunks = np.array_split(np.arange(_P.n_sites), nw * 4)
    with mp.get_context("fork").Pool(nw) as pool:
        parts = pool.map(_work, [c.tolist() for c in chunks])
    I = np.sum(parts, axis=0)
    out = {
        "about": "FP64 conventional-multislice EELS map of the config-2 workload (synth.config2) at "
                 "sampled probes; written by tests/golden/make_config2_samples.py (oracle only)",
        "probes_ix_iy": PROBES_IX_IY,
        "probe_index": [iy * 64 + ix for ix, iy in PROBES_IX_IY],
        "map": [float(v) for v in I],
        "seconds": round(time.time() - t0, 1),
        "workers": nw,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config2_samples.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
