"""Batched maps of many specimens of uneven size in one captured HIP graph.

Every specimen gets its own plan, workspace (one arena, 256-byte aligned slices) and
output slice.  The first `run_eager` uploads each plan's tables into its workspace;
`capture` then records all specimens' launches (EELS_EXEC_SKIP_UPLOAD: kernels only)
into one graph, independent specimens on parallel stream branches so that their
kernels overlap on the device, with each specimen's tuned knobs set before its
launches are recorded.  `replay` launches the whole batch with one graph launch.

fused=True (split precisions): the branches run only the specimens' set-up and sweeps
(resident S-matrices), and the contractions of all specimens follow on one stream, level
by level, each level's GEMMs one grouped launch over every specimen's sites
(eels_batch_contract).
"""
from __future__ import annotations

from typing import List, Optional, Sequence

import numpy as np

from . import autotune, eels


def _align(n: int, a: int = 256) -> int:
    return (n + a - 1) // a * a


class Batch:
    def __init__(self, problems: Sequence, precision: str = "fp32", n_streams: int = 4, device: str = "cuda",
                 tuned: bool = True, fused: bool = False):
        import torch
        self.torch = torch
        self.device = device
        self.problems = list(problems)
        self.fused = fused
        # the fused contraction groups the per-transition products of all specimens, so its
        # plans use that form of the detector sum (tuning key 6 = 0; the process-wide knob is
        # set while the plans are built, so no other thread may build plans meanwhile)
        keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 0 if fused else keep)
        try:
            self.plans = [eels.Plan(p, precision=precision, resident_s=fused) for p in self.problems]
        finally:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
        if tuned:
            self.plans = [autotune.tuned_plan(pl) for pl in self.plans]
        self.tuned = tuned
        self.inputs = [eels.device_inputs(p, device) for p in self.problems]
        sizes = [_align(pl.workspace_bytes) for pl in self.plans]
        self.ws_offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        self.arena = torch.empty(int(self.ws_offsets[-1]), dtype=torch.uint8, device=device)
        if self.arena.data_ptr() % 256:
            raise eels.EelsError(4, "arena not 256-byte aligned")
        self.workspaces = [self.arena[int(self.ws_offsets[i]):int(self.ws_offsets[i + 1])]
                           for i in range(len(self.plans))]
        self.map_offsets = np.concatenate([[0], np.cumsum([pl.n_probes for pl in self.plans])]).astype(np.int64)
        self.maps = torch.zeros(int(self.map_offsets[-1]), dtype=torch.float64, device=device)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max(1, n_streams))]
        self.graph = None
        self.contraction = None
        if fused:
            self.contraction = eels.FusedContraction(self.plans, self.ws_offsets[:-1], int(self.ws_offsets[-1]))
            self.table = torch.empty(self.contraction.table_bytes, dtype=torch.uint8, device=device)
            self._table_uploaded = False
        # larger specimens first, dealt round-robin to the streams
        self.order = sorted(range(len(self.plans)), key=lambda i: -self.plans[i].workspace_bytes)

    def out(self, i: int):
        return self.maps[int(self.map_offsets[i]):int(self.map_offsets[i + 1])]

    def tune(self, reps: int = 1):
        """Autotune each distinct shape key once (cached across processes), then rebuild the
        plans whose key chose other macro tiles (same workspace size)."""
        seen = set()
        for i, pl in enumerate(self.plans):
            k = autotune.key_of(pl)
            if k not in seen:
                seen.add(k)
                autotune.tune(pl, *self.inputs[i], reps=reps)
        for i, pl in enumerate(self.plans):
            p2 = autotune.tuned_plan(pl)
            if p2 is not pl:
                if p2.workspace_bytes > self.workspaces[i].numel():
                    raise eels.EelsError(4, "retuned plan needs a larger workspace")
                self.plans[i] = p2
        if self.contraction is not None:
            self.contraction = eels.FusedContraction(self.plans, self.ws_offsets[:-1], int(self.ws_offsets[-1]))
            self.table = self.torch.empty(self.contraction.table_bytes, dtype=self.torch.uint8, device=self.device)
            self._table_uploaded = False
        self.tuned = True

    def _enqueue(self, flags: int):
        torch = self.torch
        main = torch.cuda.current_stream(self.device)
        if self.fused:
            if not self._table_uploaded:
                self.contraction.upload(self.table, stream=main)   # once, before any capture
                self._table_uploaded = True
            flags |= eels.EXEC_SWEEPS_ONLY
        for s in self.streams:
            s.wait_stream(main)
        for n, i in enumerate(self.order):
            s = self.streams[n % len(self.streams)]
            if self.tuned:
                autotune.apply(self.plans[i])
            with torch.cuda.stream(s):
                V, H = self.inputs[i]
                self.plans[i].execute(V, H, self.out(i), self.workspaces[i], stream=s, flags=flags)
        for s in self.streams:
            main.wait_stream(s)
        autotune.set_knobs(autotune.DEFAULTS)
        if self.fused:
            self.contraction.contract(self.arena, self.table, [h for _, h in self.inputs],
                                      [self.out(i) for i in range(len(self.plans))], stream=main)

    def run_eager(self):
        """Enqueue every specimen (uploading the tables); returns without waiting."""
        self._enqueue(0)

    def capture(self):
        """Record all specimens' kernels into one HIP graph (tables must be uploaded)."""
        torch = self.torch
        self.run_eager()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream(device=self.device)
        with torch.cuda.graph(g, stream=cap):
            self._enqueue(eels.EXEC_SKIP_UPLOAD)
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()

    def maps_host(self) -> List[np.ndarray]:
        self.torch.cuda.synchronize()
        m = self.maps.cpu().numpy()
        return [m[int(self.map_offsets[i]):int(self.map_offsets[i + 1])].copy() for i in range(len(self.plans))]
