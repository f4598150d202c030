"""Project autotuner for the contraction kernels.

A tuning key describes the shape class of a plan (grid, beam counts, contraction
length, order, precision, probe count bucket).  For a key not in the cache the tuner
times candidate knob settings on the real problem (one warm-up and `reps` timed
executions, HIP events on the stream) and stores the fastest in a JSON cache
(default ~/.cache/eels/tune.json, or $EELS_TUNE_CACHE).  Two stages: first the GEMM
macro-tile shapes, plan-time knobs (256- or 128-row tiles of the first and of the second
split GEMM; the plan is rebuilt for each), then, with the best shapes, the launch-time
knobs (LDS pipeline depth, tile order).  `plan_knobs` gives a key's tile shapes for
building its plans; `apply` sets a key's launch-time knobs before its launches are
enqueued or captured (they are read at launch time).
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
PLAN_KNOBS = {
    "gemm1_rows": (eels.TUNE_GEMM1_ROWS, (1, 0)),
    "gemm2_rows": (eels.TUNE_GEMM2_ROWS, (1, 0)),
}
DEFAULTS = {"sc_stages": 2, "tile_order": 2}
PLAN_DEFAULTS = {"gemm1_rows": 1, "gemm2_rows": 1}
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
        key = KNOBS[name][0] if name in KNOBS else PLAN_KNOBS[name][0]
        eels.tune_set(key, int(val))


def plan_candidates(plan: "eels.Plan") -> List[Dict[str, int]]:
    """Macro-tile shapes to try (split precision only; FP32 has one shape)."""
    if plan.precision == "fp32":
        return [dict(PLAN_DEFAULTS)]
    return [dict(zip(PLAN_KNOBS, vals)) for vals in itertools.product(*(v[1] for v in PLAN_KNOBS.values()))]


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


def _time(plan: "eels.Plan", V, H, out, ws, reps: int) -> float:
    import torch
    plan.execute(V, H, out, ws)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        plan.execute(V, H, out, ws)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(plan: "eels.Plan", V, H, reps: int = 2, force: bool = False) -> Tuple[Dict[str, int], Dict[str, float]]:
    """Time the candidates on this plan's request (macro tiles, then launch knobs); cache and
    return the best setting (plan-time and launch-time knobs) and the timings."""
    import torch
    key = key_of(plan)
    with _lock:
        cache = load_cache()
        if key in cache and not force:
            return cache[key], {}
    out = torch.empty(plan.n_probes, dtype=torch.float64, device=V.device)
    times: Dict[str, float] = {}
    set_knobs(DEFAULTS)
    best_pc, best_plan, best_ms = None, None, float("inf")
    for pc in plan_candidates(plan):
        set_knobs(pc)
        p2 = plan.replan()
        ws = p2.alloc_workspace()
        ms = _time(p2, V, H, out, ws, reps)
        times[json.dumps({**pc, **DEFAULTS}, sort_keys=True)] = ms
        if ms < best_ms:
            best_pc, best_plan, best_ms = pc, p2, ms
        del ws
    set_knobs(PLAN_DEFAULTS)
    ws = best_plan.alloc_workspace()
    best = {**best_pc, **DEFAULTS}
    for cfg in candidates(plan):
        if cfg == DEFAULTS:
            continue                            # timed in the first stage
        set_knobs(cfg)
        ms = _time(best_plan, V, H, out, ws, reps)
        times[json.dumps({**best_pc, **cfg}, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = {**best_pc, **cfg}, ms
    set_knobs(DEFAULTS)
    with _lock:
        cache = load_cache()
        cache[key] = best
        save_cache(cache)
    return best, times


def plan_knobs(plan: "eels.Plan") -> Dict[str, int]:
    """The cached macro-tile shapes of the plan's key (the defaults if never tuned)."""
    cfg = load_cache().get(key_of(plan), {})
    return {k: int(cfg.get(k, v)) for k, v in PLAN_DEFAULTS.items()}


def tuned_plan(plan: "eels.Plan") -> "eels.Plan":
    """The plan rebuilt with its key's cached macro-tile shapes (the same plan if they are the
    defaults)."""
    pk = plan_knobs(plan)
    if pk == PLAN_DEFAULTS:
        return plan
    set_knobs(pk)
    try:
        return plan.replan()
    finally:
        set_knobs(PLAN_DEFAULTS)


def apply(plan: "eels.Plan") -> Dict[str, int]:
    """Set the cached launch-time knobs of the plan's key (the defaults if it was never
    tuned); the macro-tile shapes are fixed when a plan is built (see plan_knobs)."""
    cached = load_cache().get(key_of(plan), {})
    cfg = {k: int(cached.get(k, v)) for k, v in DEFAULTS.items()}
    set_knobs(cfg)
    return cfg
