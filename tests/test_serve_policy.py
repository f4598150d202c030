"""Host-only tests of the server's admission policy (eels_admission_*, no GPU; fake footprints).
The dispatcher's recovery from a failed request is tested on the GPU
(test_gpu_batch_serve.py::test_server_recovers_from_a_failed_request)."""
import pytest

from paper_1908_07628_amd import eels


def _adm(*a, **k):
    try:
        eels.load_library()
    except ImportError as e:  # library not built
        pytest.skip(str(e))
    from paper_1908_07628_amd.serve import Admission
    return Admission(*a, **k)


def test_first_fit_within_budget_and_slots():
    pol = _adm(budget_bytes=100, max_slots=2)
    for t, fp in [(1, 60), (2, 50), (3, 30)]:
        assert pol.offer(t, fp, arrival=float(t))
    assert pol.admit(100) == [1, 3]          # 2 does not fit next to 1; 3 does
    assert pol.used == 90
    assert pol.admit(100) == []              # both slots busy
    pol.finish(1)
    assert pol.admit(100) == [2]
    assert pol.used == 80


def test_over_budget_request_is_rejected():
    pol = _adm(budget_bytes=100, max_slots=4)
    assert not pol.offer(1, 101, arrival=0.0)
    assert pol.offer(2, 100, arrival=0.0)
    assert pol.admit(100) == [2]


def test_starvation_bound_blocks_overtaking():
    pol = _adm(budget_bytes=100, max_slots=8, max_overtake=2)
    pol.offer(1, 90, 0.0)
    assert pol.admit(100) == [1]
    pol.offer(2, 80, 1.0)                     # waits for 1
    for k in range(3, 8):
        pol.offer(k, 5, float(k))
    adm = pol.admit(100)                      # small ones overtake 2 at most twice
    assert 2 not in adm and len(adm) == 2
    assert pol.admit(100) == []               # head (2) now blocks the rest
    pol.finish(1)
    for t in adm:
        pol.finish(t)
    assert pol.admit(100)[0] == 2


def test_capacity_below_the_budget_defers_admission():
    # the server passes the budget less what busy resident workspaces hold
    pol = _adm(budget_bytes=100, max_slots=2)
    pol.offer(1, 50, 0.0)
    assert pol.admit(30) == []
    assert pol.admit(60) == [1]


def test_cancel_queued_and_finish_unknown():
    pol = _adm(budget_bytes=10, max_slots=1)
    pol.offer(1, 10, 0.0)
    pol.offer(2, 10, 1.0)
    assert pol.admit(10) == [1]
    assert pol.cancel(2)
    assert not pol.cancel(2)                  # no longer queued
    assert not pol.cancel(1)                  # running, not queued
    pol.finish(1)
    pol.finish(1)                             # finishing twice changes nothing
    assert pol.used == 0
    assert pol.admit(10) == []
