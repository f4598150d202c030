"""ctypes binding of libeels.so (argument marshalling only).

Every step of the EELS map runs in the library's HIP kernels; PyTorch provides the
device buffers and the stream.  A missing library raises: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Any, Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeels.so")

FP32, BF16_SPLIT, FP16_SPLIT = 0, 1, 2
ORDER_AUTO, ORDER_S_FIRST, ORDER_PROBE_FIRST = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16_split": BF16_SPLIT, "fp16_split": FP16_SPLIT}
ORDERS = {"auto": ORDER_AUTO, "s_first": ORDER_S_FIRST, "probe_first": ORDER_PROBE_FIRST}
DETSUMS = {"auto": 0, "direct": 1, "gram": 2}

STATUS = {0: "ok", 1: "invalid argument", 2: "band limit", 3: "unsupported size", 4: "workspace",
          5: "out of memory budget", 6: "device error", 7: "cancelled", 8: "internal"}


class EelsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"eels status {status} ({STATUS.get(status, '?')}): {msg}")
        self.status = status


class Site(C.Structure):
    _fields_ = [("slice", C.c_int), ("n_trans", C.c_int), ("x_A", C.c_double), ("y_A", C.c_double),
                ("h_offset", C.c_int64)]


class ProblemC(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("lx_A", C.c_double), ("ly_A", C.c_double),
                ("n_slices", C.c_int), ("dz_A", C.POINTER(C.c_double)), ("energy_eV", C.c_double),
                ("lambda_A", C.c_double), ("sigma", C.c_double), ("aperture_mrad", C.c_double),
                ("det_inner_mrad", C.c_double), ("det_outer_mrad", C.c_double), ("defocus_A", C.c_double),
                ("cs_A", C.c_double), ("interp_f", C.c_int), ("bandlimit", C.c_double),
                ("window_A", C.c_double), ("n_probes", C.c_int), ("probe_xy", C.POINTER(C.c_double)),
                ("n_sites", C.c_int), ("sites", C.POINTER(Site)), ("n_trans_total", C.c_int64),
                ("precision", C.c_int), ("order", C.c_int), ("max_workspace_bytes", C.c_size_t),
                ("real_space", C.c_int), ("resident_s", C.c_int), ("detector_sum", C.c_int),
                ("s1_mode", C.c_int), ("n_images", C.c_int), ("image_detectors_mrad", C.POINTER(C.c_double))]


class PlanInfo(C.Structure):
    _fields_ = [("n_beams_in", C.c_int), ("n_beams_out", C.c_int), ("n_beams_in_fine", C.c_int),
                ("n_live_x", C.c_int), ("window_nx", C.c_int), ("window_ny", C.c_int), ("k_pixels", C.c_int),
                ("k_stride", C.c_int), ("n_ion_slices", C.c_int), ("n_groups", C.c_int), ("n_batches", C.c_int),
                ("order", C.c_int), ("band_basis", C.c_int), ("band_pixels", C.c_int),
                ("lambda_A", C.c_double), ("sigma", C.c_double), ("gemm_flops", C.c_double),
                ("sweep_bytes", C.c_double), ("sweep_beam_slices", C.c_double), ("workspace_bytes", C.c_size_t),
                ("gram_form", C.c_int), ("window_gram_form", C.c_int), ("raster_form", C.c_int),
                ("n_checkpoints", C.c_int)]


class RequestTiming(C.Structure):
    _fields_ = [("arrival_s", C.c_double), ("start_s", C.c_double), ("finish_s", C.c_double),
                ("resident_hit", C.c_int), ("status", C.c_int), ("workspace_bytes", C.c_size_t)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("failed", C.c_int64),
                ("cancelled", C.c_int64), ("resident_hits", C.c_int64), ("evictions", C.c_int64),
                ("resident_bytes", C.c_size_t), ("resident_entries", C.c_int64), ("running_bytes", C.c_size_t)]


_LIB: Optional[C.CDLL] = None

EXPORTS = ["eels_get_version", "eels_status_string", "eels_last_error", "eels_plan_create",
           "eels_plan_workspace_bytes", "eels_plan_info_get", "eels_plan_beams", "eels_plan_destroy",
           "eels_execute", "eels_debug_s1", "eels_debug_s2", "eels_gemm_work_bytes", "eels_debug_cgemm",
           "eels_tune_set", "eels_tune_get", "eels_timing_enable", "eels_timing_read", "eels_execute_ex",
           "eels_plan_s_signature", "eels_execute_images", "eels_conventional_workspace_bytes",
           "eels_conventional_map", "eels_batch_create", "eels_batch_table_bytes", "eels_batch_upload",
           "eels_batch_contract", "eels_batch_destroy", "eels_map_mean", "eels_map_ratio", "eels_server_create",
           "eels_server_submit", "eels_server_poll", "eels_server_wait", "eels_server_cancel", "eels_server_release",
           "eels_server_get_stats", "eels_server_destroy", "eels_admission_create", "eels_admission_offer",
           "eels_admission_admit", "eels_admission_finish", "eels_admission_cancel", "eels_admission_used",
           "eels_admission_destroy", "eels_execute_noalloc"]
EXEC_SKIP_UPLOAD, EXEC_SKIP_SWEEPS, EXEC_SWEEPS_ONLY = 1, 2, 4
PHASES = ["setup", "sweep", "producer", "gemm1", "gemm2", "reduce", "images", "gram", "raster"]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"libeels.so not built ({path}); run __graft_entry__.build()")
    lib = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    lib.eels_get_version.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.eels_status_string.restype = C.c_char_p
    lib.eels_last_error.restype = C.c_char_p
    lib.eels_plan_create.argtypes = [C.POINTER(vp), C.POINTER(ProblemC)]
    lib.eels_plan_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.eels_plan_info_get.argtypes = [vp, C.POINTER(PlanInfo)]
    lib.eels_plan_beams.argtypes = [vp, C.c_int, C.POINTER(C.c_int), C.c_int]
    lib.eels_plan_destroy.argtypes = [vp]
    lib.eels_execute.argtypes = [vp, vp, vp, vp, vp, sz, vp]
    lib.eels_execute_ex.argtypes = [vp, vp, vp, vp, vp, sz, vp, C.c_uint]
    lib.eels_execute_images.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, C.c_uint]
    lib.eels_plan_s_signature.argtypes = [vp, C.POINTER(C.c_uint64)]
    lib.eels_conventional_workspace_bytes.argtypes = [vp, C.c_int]
    lib.eels_conventional_workspace_bytes.restype = sz
    lib.eels_conventional_map.argtypes = [vp, vp, vp, vp, C.c_int, vp, sz, vp]
    lib.eels_debug_s1.argtypes = [vp, vp, C.c_int, vp, vp, sz, vp]
    lib.eels_debug_s2.argtypes = [vp, vp, C.c_int, vp, vp, sz, vp]
    lib.eels_gemm_work_bytes.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.eels_gemm_work_bytes.restype = sz
    lib.eels_debug_cgemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp, C.c_int, vp, C.c_int,
                                     vp, vp, vp]
    lib.eels_batch_create.argtypes = [C.POINTER(vp), C.POINTER(vp), C.c_int, C.POINTER(sz), sz]
    lib.eels_batch_table_bytes.argtypes = [vp, C.POINTER(sz)]
    lib.eels_batch_upload.argtypes = [vp, vp, vp]
    lib.eels_batch_contract.argtypes = [vp, vp, vp, C.POINTER(vp), C.POINTER(vp), vp]
    lib.eels_batch_destroy.argtypes = [vp]
    lib.eels_execute_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.eels_map_mean.argtypes = [vp, vp, C.c_int, C.c_int64, vp]
    lib.eels_map_ratio.argtypes = [vp, vp, vp, C.c_int64, vp]
    u64 = C.c_uint64
    lib.eels_server_create.argtypes = [C.POINTER(vp), C.c_int, sz, C.c_int]
    lib.eels_server_submit.argtypes = [vp, C.POINTER(ProblemC), vp, vp, vp, C.POINTER(u64)]
    lib.eels_server_poll.argtypes = [vp, u64, C.POINTER(C.c_int), C.POINTER(RequestTiming)]
    lib.eels_server_wait.argtypes = [vp, u64, C.c_double, C.POINTER(C.c_int), C.POINTER(RequestTiming)]
    lib.eels_server_cancel.argtypes = [vp, u64]
    lib.eels_server_release.argtypes = [vp, u64]
    lib.eels_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.eels_server_destroy.argtypes = [vp]
    lib.eels_admission_create.argtypes = [C.POINTER(vp), sz, C.c_int, C.c_int]
    lib.eels_admission_offer.argtypes = [vp, u64, sz, C.c_double]
    lib.eels_admission_admit.argtypes = [vp, sz, C.POINTER(u64), C.c_int]
    lib.eels_admission_admit.restype = C.c_int
    lib.eels_admission_finish.argtypes = [vp, u64]
    lib.eels_admission_cancel.argtypes = [vp, u64]
    lib.eels_admission_used.argtypes = [vp]
    lib.eels_admission_used.restype = sz
    lib.eels_admission_destroy.argtypes = [vp]
    lib.eels_tune_set.argtypes = [C.c_int, C.c_int]
    lib.eels_tune_get.argtypes = [C.c_int]
    lib.eels_timing_enable.argtypes = [C.c_int]
    lib.eels_timing_read.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_int)]
    _LIB = lib
    return lib


def _check(st: int):
    if st != 0:
        msg = load_library().eels_last_error().decode(errors="replace")
        raise EelsError(st, msg)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def problem_struct(pr: Any, precision: str = "fp32", order: str = "auto", max_workspace_bytes: int = 0,
                   lambda_A: float = 0.0, sigma: float = 0.0, real_space: bool = False, resident_s: bool = False,
                   detector_sum: str = "auto", images=(), s1_mode: str = "stored"):
    """The C problem statement (eels_problem) of a problem object, and the arrays it points
    into (keep them alive as long as the struct is used)."""
    img = np.ascontiguousarray(np.asarray(images, dtype=np.float64).reshape(-1, 2))
    dz = np.ascontiguousarray(pr.dz, dtype=np.float64)
    probes = np.ascontiguousarray(pr.probes, dtype=np.float64).reshape(-1, 2)
    S = len(pr.site_slice)
    sites = (Site * max(S, 1))()
    for s in range(S):
        sites[s] = Site(int(pr.site_slice[s]), int(pr.site_ntrans[s]), float(pr.site_xy[s][0]),
                        float(pr.site_xy[s][1]), int(pr.site_hoff[s]))
    n_trans = int(pr.H.shape[0]) if getattr(pr, "H", None) is not None else int(
        max([int(pr.site_hoff[s]) + int(pr.site_ntrans[s]) for s in range(S)], default=0))
    pc = ProblemC(
        nx=int(pr.nx), ny=int(pr.ny), lx_A=float(pr.lx), ly_A=float(pr.ly), n_slices=len(dz),
        dz_A=dz.ctypes.data_as(C.POINTER(C.c_double)), energy_eV=float(pr.energy_eV),
        lambda_A=float(lambda_A), sigma=float(sigma), aperture_mrad=float(pr.aperture_mrad),
        det_inner_mrad=float(pr.det_inner_mrad), det_outer_mrad=float(pr.det_outer_mrad),
        defocus_A=float(getattr(pr, "defocus_A", 0.0)), cs_A=float(getattr(pr, "cs_A", 0.0)),
        interp_f=int(pr.interp_f), bandlimit=float(pr.bandlimit), window_A=float(pr.window_A),
        n_probes=int(probes.shape[0]),
        probe_xy=probes.ctypes.data_as(C.POINTER(C.c_double)), n_sites=S,
        sites=sites, n_trans_total=n_trans, precision=PRECISIONS[precision], order=ORDERS[order],
        max_workspace_bytes=int(max_workspace_bytes), real_space=int(bool(real_space)),
        resident_s=int(bool(resident_s)), detector_sum=DETSUMS[detector_sum],
        s1_mode={"stored": 0, "inverse": 1, "inverse_s2": 2}[s1_mode], n_images=int(img.shape[0]),
        image_detectors_mrad=img.ctypes.data_as(C.POINTER(C.c_double)))
    return pc, {"img": img, "dz": dz, "probes": probes, "sites": sites}


class Plan:
    """Host plan of one map request.  ``problem`` is any object with the fields of the
    problem statement (grid, cell, slices, optics, sites, probes; see include/eels.h)."""

    def __init__(self, problem: Any, precision: str = "fp32", order: str = "auto",
                 max_workspace_bytes: int = 0, lambda_A: float = 0.0, sigma: float = 0.0,
                 real_space: bool = False, resident_s: bool = False, detector_sum: str = "auto",
                 images=(), s1_mode: str = "stored"):
        """images: elastic companion-image rings [(inner_mrad, outer_mrad), ...]; outer <= 0
        means the band limit (e.g. ((0, det_outer), (60, 0)) for iBF and ADF).  s1_mode:
        "stored" (exact), "inverse" (S_1 retreated with the inverse multislice, Sec. 4.C) or
        "inverse_s2" (S_2 formed at the entrance and retreated towards the exit, as Sec. 4.C
        describes it; contracts in real space)."""
        lib = load_library()
        self._window_gram = tune_get(TUNE_WINDOW_GRAM)     # plan-time form of the detector sum
        self._source = (problem, dict(precision=precision, order=order, max_workspace_bytes=max_workspace_bytes,
                                      lambda_A=lambda_A, sigma=sigma, real_space=real_space, resident_s=resident_s,
                                      detector_sum=detector_sum, images=images, s1_mode=s1_mode))
        self.problem, self._keep = problem_struct(
            problem, precision=precision, order=order, max_workspace_bytes=max_workspace_bytes, lambda_A=lambda_A,
            sigma=sigma, real_space=real_space, resident_s=resident_s, detector_sum=detector_sum, images=images,
            s1_mode=s1_mode)
        self.n_images = int(self.problem.n_images)
        self._probes = self._keep["probes"]
        self._dz = self._keep["dz"]
        pr = problem
        self.precision = precision
        h = C.c_void_p()
        _check(lib.eels_plan_create(C.byref(h), C.byref(self.problem)))
        self._h = h
        self.n_probes = int(self._probes.shape[0])
        self.nx, self.ny, self.n_slices = int(pr.nx), int(pr.ny), len(self._dz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.eels_plan_destroy(h)
            self._h = None

    def replan(self) -> "Plan":
        """A new plan of the same request under the current plan-time tile knobs (tile rows,
        Gram stacking) and this plan's form of the detector sum.  It sets the process-wide
        knob 6 for the duration of the call, so it must not run while another thread
        creates plans."""
        problem, kw = self._source
        keep = tune_get(TUNE_WINDOW_GRAM)
        tune_set(TUNE_WINDOW_GRAM, self._window_gram)
        try:
            return Plan(problem, **kw)
        finally:
            tune_set(TUNE_WINDOW_GRAM, keep)

    @property
    def workspace_bytes(self) -> int:
        v = C.c_size_t()
        _check(load_library().eels_plan_workspace_bytes(self._h, C.byref(v)))
        return int(v.value)

    def info(self) -> Dict[str, Any]:
        inf = PlanInfo()
        _check(load_library().eels_plan_info_get(self._h, C.byref(inf)))
        return {name: getattr(inf, name) for name, _ in PlanInfo._fields_}

    def beams(self, which: int) -> np.ndarray:
        inf = self.info()
        n = inf["n_beams_in"] if which == 0 else inf["n_beams_out"]
        buf = (C.c_int * (2 * n))()
        _check(load_library().eels_plan_beams(self._h, which, buf, n))
        return np.frombuffer(buf, dtype=np.int32).reshape(n, 2).copy()

    # ------------------------------------------------------------------ device calls
    def alloc_workspace(self, device="cuda"):
        import torch
        ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)
        if ws.data_ptr() % 256:
            raise EelsError(4, "workspace allocation not 256-byte aligned")
        return ws

    def execute(self, V, H, out_map, workspace, stream=None, flags: int = 0):
        """Enqueue the map computation (device tensors; out_map float64 [P]).  flags:
        EXEC_SKIP_UPLOAD (tables already in this workspace; kernels only, graph-capturable),
        EXEC_SKIP_SWEEPS (reuse resident S-matrix data of a plan with the same signature)."""
        _check(load_library().eels_execute_ex(self._h, _ptr(V), _ptr(H), _ptr(out_map), _ptr(workspace),
                                              workspace.numel(), _stream(stream), int(flags)))

    def execute_images(self, V, H, out_map, out_images, workspace, stream=None, flags: int = 0):
        """As execute, and writes the companion images (float64 [n_images, P])."""
        _check(load_library().eels_execute_images(self._h, _ptr(V), _ptr(H), _ptr(out_map), _ptr(out_images),
                                                  _ptr(workspace), workspace.numel(), _stream(stream),
                                                  int(flags)))

    def conventional_workspace_bytes(self, probe_chunk: int) -> int:
        return int(load_library().eels_conventional_workspace_bytes(self._h, int(probe_chunk)))

    def conventional_map(self, V, H, out_map, probe_chunk: int, workspace, stream=None):
        """Enqueue the conventional multislice map (Sec. 3, first algorithm; interp_f = 1),
        probe_chunk probes at a time, into out_map (float64 [P])."""
        _check(load_library().eels_conventional_map(self._h, _ptr(V), _ptr(H), _ptr(out_map), int(probe_chunk),
                                                    _ptr(workspace), workspace.numel(), _stream(stream)))

    def conventional_chunk(self, max_bytes: int) -> int:
        """Largest probe chunk whose conventional workspace fits max_bytes (at least 1)."""
        lo, hi = 1, max(1, self.n_probes)
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if self.conventional_workspace_bytes(mid) <= max_bytes:
                lo = mid
            else:
                hi = mid - 1
        return lo

    def s_signature(self) -> int:
        v = C.c_uint64()
        _check(load_library().eels_plan_s_signature(self._h, C.byref(v)))
        return int(v.value)

    def debug_s1(self, V, slice_index: int, workspace, stream=None):
        import torch
        out = torch.empty((self.info()["n_beams_in"], self.ny, self.nx), dtype=torch.complex64, device=V.device)
        _check(load_library().eels_debug_s1(self._h, _ptr(V), int(slice_index), _ptr(out), _ptr(workspace),
                                            workspace.numel(), _stream(stream)))
        return out

    def debug_s2(self, V, slice_index: int, workspace, stream=None):
        import torch
        out = torch.empty((self.info()["n_beams_out"], self.ny, self.nx), dtype=torch.complex64, device=V.device)
        _check(load_library().eels_debug_s2(self._h, _ptr(V), int(slice_index), _ptr(out), _ptr(workspace),
                                            workspace.numel(), _stream(stream)))
        return out


class FusedContraction:
    """The contractions of several resident split-precision plans, level by level in grouped
    launches over one merged descriptor table (eels_batch_*).  The plans' workspaces are
    regions of one arena at ws_offsets (bytes)."""

    def __init__(self, plans, ws_offsets, arena_bytes: int):
        lib = load_library()
        self.plans = list(plans)                        # kept alive for the batch's lifetime
        arr = (C.c_void_p * len(self.plans))(*[pl._h.value for pl in self.plans])
        offs = (C.c_size_t * len(self.plans))(*[int(o) for o in ws_offsets])
        h = C.c_void_p()
        _check(lib.eels_batch_create(C.byref(h), arr, len(self.plans), offs, int(arena_bytes)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.eels_batch_destroy(h)
            self._h = None

    @property
    def table_bytes(self) -> int:
        v = C.c_size_t()
        _check(load_library().eels_batch_table_bytes(self._h, C.byref(v)))
        return int(v.value)

    def upload(self, table, stream=None):
        """Copy the merged descriptors into `table` (device uint8 tensor of table_bytes)."""
        _check(load_library().eels_batch_upload(self._h, _ptr(table), _stream(stream)))

    def contract(self, arena, table, H_list, maps, stream=None):
        """Enqueue the fused contractions after every plan's EXEC_SWEEPS_ONLY execute."""
        n = len(self.plans)
        hs = (C.c_void_p * n)(*[_ptr(h) for h in H_list])
        ms = (C.c_void_p * n)(*[_ptr(m) for m in maps])
        _check(load_library().eels_batch_contract(self._h, _ptr(arena), _ptr(table), hs, ms, _stream(stream)))


def device_inputs(problem, device="cuda"):
    """Upload V (float32) and H (complex64) of a problem to the device."""
    import torch
    V = torch.from_numpy(np.ascontiguousarray(problem.V, dtype=np.float32)).to(device)
    H = torch.from_numpy(np.ascontiguousarray(problem.H, dtype=np.complex64)).to(device)
    return V, H


def solve(problem, precision: str = "fp32", order: str = "auto", device="cuda",
          max_workspace_bytes: int = 0, real_space: bool = False, detector_sum: str = "auto",
          s1_mode: str = "stored") -> np.ndarray:
    """Compute one EELS map on the GPU and return it as float64 numpy [n_probes]."""
    import torch
    plan = Plan(problem, precision=precision, order=order, max_workspace_bytes=max_workspace_bytes,
                real_space=real_space, detector_sum=detector_sum, s1_mode=s1_mode)
    V, H = device_inputs(problem, device)
    ws = plan.alloc_workspace(device)
    out = torch.empty(plan.n_probes, dtype=torch.float64, device=device)
    plan.execute(V, H, out, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def solve_conventional(problem, probe_chunk: int = 0, device="cuda", max_bytes: int = 0) -> np.ndarray:
    """EELS map by conventional multislice on the GPU (interp_f = 1), float64 numpy [n_probes].
    probe_chunk 0: as many probes at a time as fit max_bytes (default: half the free
    device memory)."""
    import torch
    plan = Plan(problem)
    if probe_chunk <= 0:
        if max_bytes <= 0:
            free, _ = torch.cuda.mem_get_info()
            max_bytes = free // 2
        probe_chunk = plan.conventional_chunk(max_bytes)
    V, H = device_inputs(problem, device)
    ws = torch.empty(plan.conventional_workspace_bytes(probe_chunk), dtype=torch.uint8, device=device)
    out = torch.empty(plan.n_probes, dtype=torch.float64, device=device)
    plan.conventional_map(V, H, out, probe_chunk, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def solve_with_images(problem, images, precision: str = "fp32", device="cuda", **kw):
    """EELS map and elastic companion images of one problem: (map [P], images [n, P])."""
    import torch
    plan = Plan(problem, precision=precision, images=images, **kw)
    V, H = device_inputs(problem, device)
    ws = plan.alloc_workspace(device)
    out = torch.empty(plan.n_probes, dtype=torch.float64, device=device)
    img = torch.empty((plan.n_images, plan.n_probes), dtype=torch.float64, device=device)
    plan.execute_images(V, H, out, img, ws)
    torch.cuda.synchronize()
    return out.cpu().numpy(), img.cpu().numpy()


def map_mean(maps, out=None, stream=None):
    """Device mean over the first axis of maps (float64 [n_maps, n]) by eels_map_mean (FP64, in
    configuration order); returns out (float64 [n])."""
    import torch
    if maps.dtype != torch.float64 or maps.dim() != 2 or not maps.is_contiguous():
        raise EelsError(1, "maps must be a contiguous float64 [n_maps, n] device tensor")
    if out is None:
        out = torch.empty(maps.shape[1], dtype=torch.float64, device=maps.device)
    _check(load_library().eels_map_mean(_ptr(out), _ptr(maps), int(maps.shape[0]), int(maps.shape[1]),
                                        _stream(stream)))
    return out


def map_ratio(num, den, out=None, stream=None):
    """Device num / den where den > 0, else 0 (eels_map_ratio), float64 tensors of one length."""
    import torch
    if num.numel() != den.numel() or num.dtype != torch.float64 or den.dtype != torch.float64:
        raise EelsError(1, "num and den must be float64 tensors of one length")
    if out is None:
        out = torch.empty_like(num)
    _check(load_library().eels_map_ratio(_ptr(out), _ptr(num), _ptr(den), int(num.numel()), _stream(stream)))
    return out


def bf_corrected(eels_map, ibf, device="cuda"):
    """EELS map divided by the incoherent bright-field image of the EELS detector's angles
    (device division by eels_map_ratio; host arrays in and out)."""
    import torch
    num = torch.as_tensor(np.ascontiguousarray(eels_map, dtype=np.float64)).to(device)
    den = torch.as_tensor(np.ascontiguousarray(ibf, dtype=np.float64)).to(device)
    out = map_ratio(num, den)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def gemm_work_bytes(m: int, n: int, k: int) -> int:
    return int(load_library().eels_gemm_work_bytes(m, n, k))


TUNE_SC_STAGES = 0
TUNE_TILE_ORDER = 1
TUNE_SC_SCHED = 2
TUNE_GRAM_STACK = 3
TUNE_GEMM1_ROWS = 4
TUNE_GEMM2_ROWS = 5
TUNE_WINDOW_GRAM = 6
TUNE_RASTER = 7
TUNE_CHECKPOINT = 8
TUNE_WG_FUSED = 9
TUNE_GRAM_ROWS = 10
TUNE_GEMM_STAGING = 11


def tune_set(key: int, value: int):
    _check(load_library().eels_tune_set(int(key), int(value)))


def tune_get(key: int) -> int:
    return int(load_library().eels_tune_get(int(key)))


def timing_enable(capacity: int = 4096):
    """Record HIP events around the launch groups of every eels_execute (diagnostics)."""
    _check(load_library().eels_timing_enable(int(capacity)))


def timing_read() -> Dict[str, Any]:
    """Per-phase milliseconds and group counts of the most recent execute (synchronises)."""
    ms = (C.c_double * len(PHASES))()
    cnt = (C.c_int * len(PHASES))()
    _check(load_library().eels_timing_read(ms, cnt))
    return {ph: {"ms": ms[i], "count": cnt[i]} for i, ph in enumerate(PHASES)}


def cgemm(A, B, precision: str = "fp32", norm2: bool = False, stream=None):
    """C = A @ B.T for complex64 device tensors A [m, k], B [n, k] through the contraction
    kernels; with norm2 returns sum_m |C[m, n]|^2 (float64 [n])."""
    import torch
    m, k = A.shape
    n, k2 = B.shape
    assert k == k2 and A.dtype == torch.complex64 and B.dtype == torch.complex64
    lda = ldb = k + (k & 1)
    Ap = torch.zeros((m, lda), dtype=torch.complex64, device=A.device)
    Ap[:, :k] = A
    Bp = torch.zeros((n, ldb), dtype=torch.complex64, device=B.device)
    Bp[:, :k] = B
    work = torch.empty(gemm_work_bytes(m, n, k), dtype=torch.uint8, device=A.device)
    if norm2:
        out = torch.empty(n, dtype=torch.float64, device=A.device)
        _check(load_library().eels_debug_cgemm(PRECISIONS[precision], m, n, k, _ptr(Ap), lda, _ptr(Bp), ldb, None,
                                               0, _ptr(out), _ptr(work), _stream(stream)))
    else:
        out = torch.empty((m, n), dtype=torch.complex64, device=A.device)
        _check(load_library().eels_debug_cgemm(PRECISIONS[precision], m, n, k, _ptr(Ap), lda, _ptr(Bp), ldb,
                                               _ptr(out), n, None, _ptr(work), _stream(stream)))
    return out
