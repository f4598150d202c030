"""The allocation-free entry point (eels_execute_noalloc) called through the C ABI: two calls
in a row, the second with a smaller problem, each against eels_execute of the same plan with a
caller-owned workspace (bitwise equal) and against the oracle; a plan larger than the fixed
scratch is refused."""
import ctypes as C

import numpy as np
import pytest

from maptol import maps_close
import synth
from oracle import prism

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run_both(eels, p, precision):
    lib = eels.load_library()
    plan = eels.Plan(p, precision=precision)
    V, H = eels.device_inputs(p)
    ws = plan.alloc_workspace()
    ref = torch.empty(plan.n_probes, dtype=torch.float64, device="cuda")
    plan.execute(V, H, ref, ws)
    got = torch.full((plan.n_probes,), -1.0, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    st = lib.eels_execute_noalloc(plan._h, C.c_void_p(V.data_ptr()), C.c_void_p(H.data_ptr()),
                                  C.c_void_p(got.data_ptr()), C.c_void_p(stream))
    assert st == 0, lib.eels_last_error()
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_noalloc_matches_execute_on_two_calls(precision, tol):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    big = synth.config1()                                    # about 70 MiB of workspace
    small = synth.random_problem(3, n=32, L=8.0, nz=3)        # about 6 MiB
    for p in (big, small):
        print("noalloc", precision, p.nx, flush=True)
        got, ref = _run_both(eels, p, precision)
        assert np.array_equal(got, ref)
        assert maps_close(got, prism.prism_map(p), tol)


def test_noalloc_refuses_a_plan_beyond_its_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    lib = eels.load_library()
    p = synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=4, f=2)
    plan = eels.Plan(p, precision="bf16_split")
    assert plan.workspace_bytes > (128 << 20)
    st = lib.eels_execute_noalloc(plan._h, C.c_void_p(0), C.c_void_p(0), C.c_void_p(0), C.c_void_p(0))
    assert st == 4                                           # EELS_ERR_WORKSPACE, before any device work
    assert b"eels_execute_noalloc holds at most" in lib.eels_last_error()
