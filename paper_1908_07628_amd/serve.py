"""Serving loop for EELS-map requests on one GPU (continuous batching).

Requests arrive at any time (`submit`).  A dispatcher thread admits them while a slot
(stream) is free and their memory footprint (plan workspace + inputs) fits the HBM
budget; admitted requests run concurrently on their own streams, so work of requests
that arrive while others are on the GPU overlaps on the device.  Completion is
detected with stream events; latency = completion - arrival.

S-matrix residency: a completed request's workspace keeps its S-matrix data (plans are
built with resident_s).  A later request for the same specimen and sites (same V, H
content and the same S signature) reuses it with EELS_EXEC_SKIP_SWEEPS: only the probe
coefficients and the contractions run.  Resident workspaces count against the budget and
are evicted least-recently-used when an admission needs the memory.

`AdmissionPolicy` holds the pure host decision logic (testable without a GPU).
"""
from __future__ import annotations

import collections
import dataclasses
import hashlib
import threading
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Tuple

import numpy as np

from . import eels


@dataclasses.dataclass
class Pending:
    ticket: int
    footprint: int
    arrival: float
    skipped: int = 0


class AdmissionPolicy:
    """First-fit admission in arrival order with an anti-starvation bound: once the oldest
    queued request has been overtaken `max_overtake` times, nothing behind it is admitted
    until it fits.  A request larger than the whole budget is rejected."""

    def __init__(self, budget_bytes: int, max_slots: int, max_overtake: int = 4):
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.max_overtake = int(max_overtake)
        self.queue: Deque[Pending] = collections.deque()
        self.used = 0
        self.running: Dict[int, int] = {}

    def offer(self, ticket: int, footprint: int, arrival: float) -> bool:
        if footprint > self.budget:
            return False
        self.queue.append(Pending(ticket, int(footprint), float(arrival)))
        return True

    def cancel(self, ticket: int) -> bool:
        for p in list(self.queue):
            if p.ticket == ticket:
                self.queue.remove(p)
                return True
        return False

    def admit(self, reclaimable: int = 0) -> List[int]:
        """Tickets to start now.  `reclaimable` bytes can be freed on demand (resident data)."""
        out = []
        head_blocked = False
        for p in list(self.queue):
            if len(self.running) >= self.max_slots:
                break
            fits = self.used + p.footprint <= self.budget + reclaimable
            if fits and not head_blocked:
                self.queue.remove(p)
                self.running[p.ticket] = p.footprint
                self.used += p.footprint
                out.append(p.ticket)
                for q in self.queue:
                    if q.arrival < p.arrival:
                        q.skipped += 1
            elif not fits and p is self.queue[0] and p.skipped >= self.max_overtake:
                head_blocked = True
        return out

    def finish(self, ticket: int):
        fp = self.running.pop(ticket, 0)
        self.used -= fp


@dataclasses.dataclass
class Result:
    ticket: int
    done: bool = False
    error: Optional[str] = None
    map: Optional[np.ndarray] = None
    arrival: float = 0.0
    start: float = 0.0
    finish: float = 0.0
    resident_hit: bool = False

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def specimen_key(problem) -> str:
    h = hashlib.blake2b(digest_size=16)
    h.update(np.ascontiguousarray(problem.V).view(np.uint8).data)
    h.update(np.ascontiguousarray(problem.H).view(np.uint8).data)
    return h.hexdigest()


class Server:
    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, precision: str = "fp32",
                 residency: bool = True, device: str = "cuda", clock: Callable[[], float] = time.perf_counter):
        import torch
        self.torch = torch
        self.device = device
        self.precision = precision
        self.residency = residency
        self.clock = clock
        self.policy = AdmissionPolicy(hbm_budget_bytes, max_slots)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(max_slots)]
        self.free_streams = list(range(max_slots))
        self.lock = threading.Lock()
        self.cv = threading.Condition(self.lock)
        self.requests: Dict[int, Dict[str, Any]] = {}
        self.results: Dict[int, Result] = {}
        self.resident: "collections.OrderedDict[Tuple[str, int], Dict[str, Any]]" = collections.OrderedDict()
        self.next_ticket = 1
        self.stop_flag = False
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # ------------------------------------------------------------------ client API
    def submit(self, problem, key: Optional[str] = None, arrival: Optional[float] = None) -> int:
        plan = eels.Plan(problem, precision=self.precision, resident_s=self.residency)
        inputs_bytes = int(np.asarray(problem.V).nbytes + np.asarray(problem.H).nbytes)
        footprint = plan.workspace_bytes + inputs_bytes + 8 * plan.n_probes
        with self.cv:
            t = self.next_ticket
            self.next_ticket += 1
            arr = self.clock() if arrival is None else arrival
            self.results[t] = Result(t, arrival=arr)
            if not self.policy.offer(t, footprint, arr):
                self.results[t].done = True
                self.results[t].error = "footprint exceeds the HBM budget"
                return t
            key = key if key is not None else (specimen_key(problem) if self.residency else "")
            self.requests[t] = {"problem": problem, "plan": plan, "key": (key, plan.s_signature()),
                                "footprint": footprint}
            self.cv.notify()
        return t

    def poll(self, ticket: int) -> Result:
        with self.lock:
            return self.results[ticket]

    def wait(self, ticket: int, timeout: float = 600.0) -> Result:
        t_end = time.perf_counter() + timeout
        with self.cv:
            while not self.results[ticket].done:
                left = t_end - time.perf_counter()
                if left <= 0:
                    raise TimeoutError(f"request {ticket}")
                self.cv.wait(min(left, 0.05))
            return self.results[ticket]

    def cancel(self, ticket: int) -> bool:
        with self.cv:
            if self.policy.cancel(ticket):
                r = self.results[ticket]
                r.done, r.error = True, "cancelled"
                self.requests.pop(ticket, None)
                return True
            return False

    def close(self):
        with self.cv:
            self.stop_flag = True
            self.cv.notify()
        self.thread.join()

    # ------------------------------------------------------------------ dispatcher
    def _resident_bytes(self) -> int:
        return sum(e["bytes"] for e in self.resident.values() if not e["busy"])

    def _evict_for(self, need: int):
        while self.resident and self.policy.used + self._resident_total() + need > self.policy.budget:
            for k, e in self.resident.items():
                if not e["busy"]:
                    self.resident.pop(k)
                    break
            else:
                return

    def _resident_total(self) -> int:
        return sum(e["bytes"] for e in self.resident.values())

    def _start(self, t: int):
        torch = self.torch
        req = self.requests[t]
        plan, prob = req["plan"], req["problem"]
        sid = self.free_streams.pop()
        st = self.streams[sid]
        res = self.resident.get(req["key"]) if self.residency else None
        hit = res is not None and not res["busy"] and res["ws"].numel() >= plan.workspace_bytes
        r = self.results[t]
        r.start = self.clock()
        with torch.cuda.stream(st):
            if hit:
                res["busy"] = True
                self.resident.move_to_end(req["key"])
                V, H, ws = res["V"], res["H"], res["ws"]
                flags = eels.EXEC_SKIP_SWEEPS
            else:
                if res is not None and not res["busy"]:
                    self.resident.pop(req["key"])
                self._evict_for(req["footprint"])
                V, H = eels.device_inputs(prob, self.device)
                ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=self.device)
                flags = 0
            out = torch.empty(plan.n_probes, dtype=torch.float64, device=self.device)
            plan.execute(V, H, out, ws, stream=st, flags=flags)
            host = torch.empty(plan.n_probes, dtype=torch.float64, pin_memory=True)
            host.copy_(out, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        req.update({"sid": sid, "event": ev, "host": host, "V": V, "H": H, "ws": ws, "out": out, "hit": hit})
        r.resident_hit = hit

    def _complete(self, t: int):
        req = self.requests.pop(t)
        r = self.results[t]
        r.map = req["host"].numpy().copy()
        r.finish = self.clock()
        r.done = True
        self.policy.finish(t)
        self.free_streams.append(req["sid"])
        if self.residency:
            key = req["key"]
            if req["hit"]:
                self.resident[key]["busy"] = False
            else:
                self.resident[key] = {"V": req["V"], "H": req["H"], "ws": req["ws"], "busy": False,
                                      "bytes": req["footprint"]}
                self._evict_for(0)

    def _loop(self):
        with self.cv:
            while True:
                if self.stop_flag and not self.requests:
                    return
                # completions
                for t, req in list(self.requests.items()):
                    if "event" in req and req["event"].query():
                        self._complete(t)
                        self.cv.notify_all()
                # admissions (resident data can be evicted to make room)
                for t in self.policy.admit(reclaimable=self._resident_bytes()):
                    try:
                        self._start(t)
                    except Exception as e:  # report the failure on the ticket
                        self.policy.finish(t)
                        self.requests.pop(t, None)
                        r = self.results[t]
                        r.done, r.error, r.finish = True, repr(e), self.clock()
                        self.cv.notify_all()
                self.cv.wait(0.002)

    # ------------------------------------------------------------------ statistics
    def latency_stats(self, tickets: Optional[List[int]] = None) -> Dict[str, float]:
        rs = [self.results[t] for t in (tickets or list(self.results)) if self.results[t].done
              and self.results[t].error is None]
        lat = np.array([r.latency for r in rs]) if rs else np.zeros(1)
        return {"n": len(rs), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                "mean_s": float(lat.mean()), "resident_hits": int(sum(r.resident_hit for r in rs))}
