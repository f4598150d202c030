"""Serving EELS-map requests on one GPU: a thin binding of the library's server.

Admission (first fit by HBM footprint, anti-starvation), the per-request streams, completion
events, S-matrix residency (workspaces kept and reused for the same V, H and S signature) and
eviction all run in libeels.so (eels_server_*, include/eels.h).  This module only marshals:
it uploads each request's inputs with torch, hands the device pointers to the server, keeps the
tensors alive until the request is done, and reads the map and the timing back.

`Admission` binds the server's admission policy on its own (eels_admission_*, host only).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Dict, List, Optional

import numpy as np

from . import eels


@dataclasses.dataclass
class Result:
    ticket: int
    done: bool = False
    error: Optional[str] = None
    status: int = 0
    map: Optional[np.ndarray] = None
    arrival: float = 0.0
    start: float = 0.0
    finish: float = 0.0
    resident_hit: bool = False
    workspace_bytes: int = 0

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class Server:
    """One GPU's request server.  submit() returns a ticket; wait()/poll() return a Result."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, precision: str = "fp32", device: str = "cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.precision = precision
        idx = self.device.index if self.device.index is not None else torch.cuda.current_device()
        h = C.c_void_p()
        eels._check(eels.load_library().eels_server_create(C.byref(h), int(idx), int(hbm_budget_bytes),
                                                           int(max_slots)))
        self._h = h
        self._live: Dict[int, tuple] = {}          # ticket -> (V, H, out, problem struct, arrays)
        self.results: Dict[int, Result] = {}

    def submit(self, problem, **plan_kw) -> int:
        """Queue one request (raises EelsError if it cannot be planned or exceeds the budget)."""
        torch = self.torch
        pc, keep = eels.problem_struct(problem, precision=self.precision, **plan_kw)
        V, H = eels.device_inputs(problem, self.device)
        out = torch.empty(int(pc.n_probes), dtype=torch.float64, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()     # inputs written before the server reads them
        t = C.c_uint64()
        eels._check(eels.load_library().eels_server_submit(self._h, C.byref(pc), eels._ptr(V), eels._ptr(H),
                                                           eels._ptr(out), C.byref(t)))
        self._live[t.value] = (V, H, out, pc, keep)
        self.results[t.value] = Result(t.value)
        return t.value

    def _finish(self, ticket: int, done: int, tm: "eels.RequestTiming") -> Result:
        r = self.results[ticket]
        r.arrival, r.start, r.finish = tm.arrival_s, tm.start_s, tm.finish_s
        r.resident_hit, r.status, r.workspace_bytes = bool(tm.resident_hit), int(tm.status), int(tm.workspace_bytes)
        if done and not r.done:
            r.done = True
            V, H, out, _, _ = self._live.pop(ticket)
            if r.status == 0:
                r.map = out.cpu().numpy()
            else:
                r.error = eels.load_library().eels_status_string(r.status).decode()
            eels.load_library().eels_server_release(self._h, C.c_uint64(ticket))
        return r

    def poll(self, ticket: int) -> Result:
        r = self.results[ticket]
        if r.done:
            return r
        done, tm = C.c_int(), eels.RequestTiming()
        eels._check(eels.load_library().eels_server_poll(self._h, C.c_uint64(ticket), C.byref(done), C.byref(tm)))
        return self._finish(ticket, done.value, tm)

    def wait(self, ticket: int, timeout: float = 600.0) -> Result:
        r = self.results[ticket]
        if r.done:
            return r
        done, tm = C.c_int(), eels.RequestTiming()
        eels._check(eels.load_library().eels_server_wait(self._h, C.c_uint64(ticket), float(timeout),
                                                         C.byref(done), C.byref(tm)))
        if not done.value:
            raise TimeoutError(f"request {ticket}")
        return self._finish(ticket, done.value, tm)

    def cancel(self, ticket: int) -> bool:
        st = eels.load_library().eels_server_cancel(self._h, C.c_uint64(ticket))
        if st == 0:
            self.poll(ticket)
        return st == 0

    def stats(self) -> Dict[str, int]:
        s = eels.ServerStats()
        eels._check(eels.load_library().eels_server_get_stats(self._h, C.byref(s)))
        return {name: int(getattr(s, name)) for name, _ in eels.ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            eels._check(eels.load_library().eels_server_destroy(self._h))
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def latency_stats(self, tickets: Optional[List[int]] = None) -> Dict[str, float]:
        rs = [self.results[t] for t in (tickets or list(self.results))
              if self.results[t].done and self.results[t].error is None]
        lat = np.array([r.latency for r in rs]) if rs else np.zeros(1)
        return {"n": len(rs), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "resident_hits": int(sum(r.resident_hit for r in rs))}


class Admission:
    """The server's admission policy (host only)."""

    def __init__(self, budget_bytes: int, max_slots: int, max_overtake: int = 4):
        h = C.c_void_p()
        eels._check(eels.load_library().eels_admission_create(C.byref(h), int(budget_bytes), int(max_slots),
                                                              int(max_overtake)))
        self._h = h
        self.max_slots = int(max_slots)

    def offer(self, ticket: int, footprint: int, arrival: float) -> bool:
        return eels.load_library().eels_admission_offer(self._h, C.c_uint64(ticket), int(footprint),
                                                        float(arrival)) == 0

    def admit(self, capacity: int) -> List[int]:
        buf = (C.c_uint64 * self.max_slots)()
        n = eels.load_library().eels_admission_admit(self._h, int(capacity), buf, self.max_slots)
        return [int(buf[i]) for i in range(n)]

    def finish(self, ticket: int):
        eels._check(eels.load_library().eels_admission_finish(self._h, C.c_uint64(ticket)))

    def cancel(self, ticket: int) -> bool:
        return eels.load_library().eels_admission_cancel(self._h, C.c_uint64(ticket)) == 0

    @property
    def used(self) -> int:
        return int(eels.load_library().eels_admission_used(self._h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            eels.load_library().eels_admission_destroy(h)
            self._h = None
