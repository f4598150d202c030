"""Frozen-phonon averaging of EELS maps.

A thermal configuration displaces every atom (and the transition potentials of the ionised
ones) by random offsets; the frozen-phonon map is the average of the maps of several seeded
configurations (the Results' nanoparticle run is one such configuration, and the runtime
discussion counts passes per configuration).  Every configuration is one full map through
the C ABI; the maps share one workspace (their plans have the same layout when the
configurations share grid, slices, sites' slices and probes), and their mean is taken on
the device by eels_map_mean.
"""
from __future__ import annotations

from typing import Sequence, Tuple

import numpy as np

from . import eels


def frozen_phonon_map(configs: Sequence, precision: str = "bf16_split", device: str = "cuda",
                      **plan_kw) -> Tuple[np.ndarray, np.ndarray]:
    """(mean map [P], per-configuration maps [n, P]) of the given configurations, which must
    share the probe positions."""
    import torch
    if not configs:
        raise ValueError("no configurations")
    P = int(np.asarray(configs[0].probes).reshape(-1, 2).shape[0])
    plans = [eels.Plan(c, precision=precision, **plan_kw) for c in configs]
    for c in configs[1:]:
        if not np.array_equal(np.asarray(c.probes), np.asarray(configs[0].probes)):
            raise ValueError("frozen-phonon configurations must share the probe positions")
    ws = torch.empty(max(pl.workspace_bytes for pl in plans), dtype=torch.uint8, device=device)
    maps = torch.empty((len(configs), P), dtype=torch.float64, device=device)
    for i, (c, pl) in enumerate(zip(configs, plans)):
        V, H = eels.device_inputs(c, device)
        pl.execute(V, H, maps[i], ws)
    mean = eels.map_mean(maps)                 # FP64 mean on the device, in configuration order
    torch.cuda.synchronize()
    return mean.cpu().numpy(), maps.cpu().numpy()
