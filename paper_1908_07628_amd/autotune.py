"""Project autotuner for the contraction kernels.

A tuning key describes the shape class of a plan (grid, beam counts, contraction
length, order, precision, probe count bucket).  For a key not in the cache the tuner
times every candidate knob setting on the real problem (one warm-up and `reps` timed
executions, HIP events on the stream) and stores the fastest in a JSON cache
(default ~/.cache/eels/tune.json, or $EELS_TUNE_CACHE).  `apply` sets the knobs of
a key before its launches are enqueued or captured (they are read at launch time).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import threading
from typing import Dict, List, Optional, Tuple

from . import eels

KNOBS = {
    "sc_stages": (eels.TUNE_SC_STAGES, (2, 3)),
    "tile_order": (eels.TUNE_TILE_ORDER, (0, 1, 2)),
}
DEFAULTS = {"sc_stages": 2, "tile_order": 2}
_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("EELS_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "eels", "tune.json"))


def key_of(plan: "eels.Plan") -> str:
    i = plan.info()
    kc = i["band_pixels"] if i["band_basis"] else i["k_pixels"]
    pb = 2 ** int(math.ceil(math.log2(max(plan.n_probes, 1))))
    return (f"{plan.nx}x{plan.ny}|N1={i['n_beams_in']}|N2={i['n_beams_out']}|K={kc}|order={i['order']}"
            f"|prec={plan.precision}|P<={pb}")


def load_cache() -> Dict[str, Dict[str, int]]:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(c: Dict[str, Dict[str, int]]):
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(c, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def set_knobs(cfg: Dict[str, int]):
    for name, val in cfg.items():
        eels.tune_set(KNOBS[name][0], int(val))


def candidates(plan: "eels.Plan") -> List[Dict[str, int]]:
    names = list(KNOBS)
    if plan.precision == "fp32":
        names = ["tile_order"]         # the pipeline depth only applies to the split GEMM
    out = []
    for vals in itertools.product(*(KNOBS[n][1] for n in names)):
        cfg = dict(DEFAULTS)
        cfg.update(dict(zip(names, vals)))
        out.append(cfg)
    return out


def tune(plan: "eels.Plan", V, H, reps: int = 2, force: bool = False) -> Tuple[Dict[str, int], Dict[str, float]]:
    """Time every candidate on this plan; cache and return the best setting and the timings."""
    import torch
    key = key_of(plan)
    with _lock:
        cache = load_cache()
        if key in cache and not force:
            return cache[key], {}
    ws = plan.alloc_workspace()
    out = torch.empty(plan.n_probes, dtype=torch.float64, device=V.device)
    times: Dict[str, float] = {}
    best, best_ms = None, float("inf")
    for cfg in candidates(plan):
        set_knobs(cfg)
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.execute(V, H, out, ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        times[json.dumps(cfg, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = cfg, ms
    set_knobs(DEFAULTS)
    with _lock:
        cache = load_cache()
        cache[key] = best
        save_cache(cache)
    return best, times


def apply(plan: "eels.Plan") -> Dict[str, int]:
    """Set the cached knobs of the plan's key (the defaults if it was never tuned)."""
    cfg = dict(DEFAULTS)
    cfg.update(load_cache().get(key_of(plan), {}))
    set_knobs(cfg)
    return cfg
