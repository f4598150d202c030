"""Host-only tests of the serving admission policy (no GPU, fake footprints)."""
from paper_1908_07628_amd.serve import AdmissionPolicy


def test_first_fit_within_budget_and_slots():
    pol = AdmissionPolicy(budget_bytes=100, max_slots=2)
    for t, fp in [(1, 60), (2, 50), (3, 30)]:
        assert pol.offer(t, fp, arrival=float(t))
    assert pol.admit() == [1, 3]            # 2 does not fit next to 1; 3 does
    assert pol.used == 90
    assert pol.admit() == []                # both slots busy
    pol.finish(1)
    assert pol.admit() == [2]
    assert pol.used == 80


def test_over_budget_request_is_rejected():
    pol = AdmissionPolicy(budget_bytes=100, max_slots=4)
    assert not pol.offer(1, 101, arrival=0.0)
    assert pol.offer(2, 100, arrival=0.0)
    assert pol.admit() == [2]


def test_starvation_bound_blocks_overtaking():
    pol = AdmissionPolicy(budget_bytes=100, max_slots=8, max_overtake=2)
    pol.offer(1, 90, 0.0)
    assert pol.admit() == [1]
    pol.offer(2, 80, 1.0)                    # waits for 1
    for k in range(3, 8):
        pol.offer(k, 5, float(k))
    adm = pol.admit()                        # small ones overtake 2 at most twice
    assert 2 not in adm and len(adm) == 2
    assert pol.admit() == []                 # head (2) now blocks the rest
    pol.finish(1)
    for t in adm:
        pol.finish(t)
    assert pol.admit()[0] == 2


def test_reclaimable_memory_allows_admission():
    pol = AdmissionPolicy(budget_bytes=100, max_slots=2)
    pol.used = 70                            # e.g. resident S-matrices
    pol.offer(1, 50, 0.0)
    assert pol.admit() == []
    assert pol.admit(reclaimable=30) == [1]


def test_cancel_queued():
    pol = AdmissionPolicy(budget_bytes=10, max_slots=1)
    pol.offer(1, 10, 0.0)
    pol.offer(2, 10, 1.0)
    assert pol.admit() == [1]
    assert pol.cancel(2)
    pol.finish(1)
    assert pol.admit() == []
