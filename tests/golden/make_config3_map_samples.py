"""Write config3_map_samples.json: FP64 PRISM map values (f = 4, 4 A crop) of the WHOLE
full-size nanoparticle workload (synth.config3: 1024 x 1024 px, 50 slices, every one of the
22,659 ionised sphere atoms x 9 transitions, N_1 = N_2 = 2025) at 64 probes spread over the
central 32 x 32 probes of the 256 x 256 raster (indices 112 .. 143 on both axes), computed
with the PRISM oracle only (oracle.prism.probe_waves_partial / intensity_partial, the same
sums as prism_map regrouped over disjoint beam sets).

Memory stays bounded: the aperture beams are swept a few at a time and each ionised slice's
probe-wave parts Psi_s are added into one shared FP64 buffer as the sweep passes the slice
(about 12 GB for the sites any sampled probe sees); the detector beams are then swept a few
at a time against the complete Psi.  Cost: about 4,000 beams x 50 slices of 1024 x 1024
FFTs plus the contractions, roughly an hour on 6 cores.

Usage: python tests/golden/make_config3_map_samples.py [n_workers]
"""
import json
import mmap
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import prism  # noqa: E402
from oracle.common import make_setup, site_eligible  # noqa: E402

N_SCAN = 256
# an 8 x 8 lattice over the central 32 x 32 probes (stride 4 px = 1.56 A)
PROBES_IX_IY = [(113 + 4 * a, 113 + 4 * b) for b in range(8) for a in range(8)]
CHUNK1, CHUNK2 = 16, 16

_G = {}


def sample_problem():
    p = synth.config3()
    idx = np.array([iy * N_SCAN + ix for ix, iy in PROBES_IX_IY])
    return p.replace(probes=p.probes[idx], probe_shape=(8, 8)), idx


def _sink(j, parts):
    psi, lock = _G["psi"], _G["locks"][j]
    with lock:
        for s, v in parts.items():
            psi[s] += v


def _psi_task(beams):
    prism.probe_waves_partial(_G["q"], beams, chunk=CHUNK1, st=_G["st"], sink=_sink)
    return len(beams)


def _int_task(beams):
    return prism.intensity_partial(_G["q"], _G["psi"], beams, chunk=CHUNK2, st=_G["st"])


def main():
    nw = int(sys.argv[1]) if len(sys.argv) > 1 else max(1, (os.cpu_count() or 2) - 2)
    t0 = time.time()
    q, idx = sample_problem()
    st = make_setup(q)
    # the sites some sampled probe sees, and their slots in one shared buffer
    K = (2 * st.win[0] + 1) * (2 * st.win[1] + 1)
    shapes, total = {}, 0
    for s in range(q.n_sites):
        ne = int(np.sum(site_eligible(q, st, s)))
        if ne:
            shapes[s] = (total, ne)
            total += K * ne
    mm = mmap.mmap(-1, max(16, 16 * total))          # anonymous, shared with the forked workers
    buf = np.frombuffer(mm, dtype=np.complex128, count=total)
    psi = {s: buf[o:o + K * ne].reshape(K, ne) for s, (o, ne) in shapes.items()}
    _G.update(q=q, st=st, psi=psi, locks={j: mp.Lock() for j in st.sites_by_slice})
    print(f"{q.n_sites} sites, {len(psi)} seen by the sampled probes; Psi {16 * total / 1e9:.1f} GB; "
          f"set-up {time.time() - t0:.0f} s", flush=True)
    n1, n2 = st.ab1.shape[0], st.ab2.shape[0]
    with mp.get_context("fork").Pool(nw) as pool:
        done = 0
        for k in pool.imap_unordered(_psi_task, [np.arange(a, min(a + CHUNK1, n1)) for a in range(0, n1, CHUNK1)]):
            done += k
            print(f"aperture beams {done}/{n1} ({time.time() - t0:.0f} s)", flush=True)
        I = np.zeros(q.n_probes)
        done = 0
        for part in pool.imap_unordered(_int_task, [np.arange(a, min(a + CHUNK2, n2)) for a in range(0, n2, CHUNK2)]):
            I += part
            done += CHUNK2
            print(f"detector beams {min(done, n2)}/{n2} ({time.time() - t0:.0f} s)", flush=True)
    out = {
        "about": "FP64 PRISM EELS map (f = 4, 4 A crop) of the whole full-size nanoparticle workload "
                 "(synth.config3, all ionised slices and sites) at 64 probes spread over the central 32 x 32 "
                 "probes of the raster; written by tests/golden/make_config3_map_samples.py (oracle only)",
        "n_sites": int(q.n_sites),
        "sites_seen": int(len(psi)),
        "probes_ix_iy": PROBES_IX_IY,
        "probe_index": [int(v) for v in idx],
        "map": [float(v) for v in I],
        "seconds": round(time.time() - t0, 1),
        "workers": nw,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config3_map_samples.json")
    json.dump(out, open(path, "w"), indent=1)
    print(json.dumps(out)[:400])


if __name__ == "__main__":
    main()
