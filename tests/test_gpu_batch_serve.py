"""GPU tests of the extensions: batched maps in a captured HIP graph, the autotuner,
S-matrix residency (EELS_EXEC_SKIP_SWEEPS) and the serving loop."""
import os
import sys

import numpy as np
import pytest

from maptol import maps_close
import synth
from oracle import metrics, prism

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    return eels


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _specimens(n=5, seed=7):
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n):
        size = [64, 128][k % 2]
        out.append(synth.random_lattice_specimen(rng, size, int(rng.integers(3, 7)), int(rng.integers(1, 4)),
                                                 nt_range=(1, 3), n_scan=int(rng.integers(4, 9)),
                                                 det_outer_mrad=30.0, name=f"b{k}"))
    return out


def test_batch_graph_replays_match_eager_and_solo():
    eels = _gpu()
    from paper_1908_07628_amd.batch import Batch
    sp = _specimens()
    b = Batch(sp, precision="fp32", n_streams=3, tuned=False)
    b.run_eager()
    eager = b.maps_host()
    for i, p in enumerate(sp):
        solo = eels.solve(p, precision="fp32")
        assert np.array_equal(eager[i], solo), i
    ref = prism.prism_map(sp[0])
    assert maps_close(eager[0], ref, 1e-4)
    b.capture()
    for rep in range(3):
        b.maps.zero_()                                  # eager work between replays
        torch.cuda.synchronize()
        b.replay()
        got = b.maps_host()
        _say("replay", rep)
        for i in range(len(sp)):
            assert np.array_equal(got[i], eager[i]), (rep, i)


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_fused_batch_contraction_matches_per_specimen(prec):
    """Fused batch: every specimen's set-up and sweeps on parallel branches, then the
    contractions of all specimens level by level, each level's GEMMs one grouped launch over
    a merged descriptor table.  Specimens of three kinds (cropped windows, f = 2 order P, and
    a full-cell band-basis cell) give launches of different epilogues in one level.  Maps
    equal each specimen's own execute bit for bit, eagerly and in three graph replays, and
    meet the split bar against the oracle."""
    eels = _gpu()
    from paper_1908_07628_amd.batch import Batch
    sp = _specimens() + [synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=4, f=2),
                         synth.random_problem(41, n=32, L=8.0, nz=3, n_sites=2, n_trans=2)]
    b = Batch(sp, precision=prec, n_streams=3, tuned=False, fused=True)
    _say("fused batch", prec, len(sp), "specimens, table bytes", b.contraction.table_bytes)
    b.run_eager()
    fused = b.maps_host()
    keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 0)       # the fused batch's form of the detector sum
        solos = [eels.solve(p, precision=prec) for p in sp]
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
    for i, solo in enumerate(solos):
        assert np.array_equal(fused[i], solo), i
    for i in (0, len(sp) - 2, len(sp) - 1):
        assert maps_close(fused[i], prism.prism_map(sp[i]), 1e-3), i
    b.capture()
    for rep in range(3):
        b.maps.zero_()                                  # eager work between replays
        torch.cuda.synchronize()
        b.replay()
        got = b.maps_host()
        _say("fused replay", rep)
        for i in range(len(sp)):
            assert np.array_equal(got[i], fused[i]), (rep, i)


GOLD4 = os.path.join(os.path.dirname(__file__), "golden", "config4_samples.json")


def test_config4_batch_sampled_probes():
    """The 64-specimen batch workload in bench.py's fused configuration (FP16 split, four
    stream branches, fused contraction in persistent launches, one captured graph, replayed):
    three of its specimens (128^2 with f = 1, 256^2 with f = 2 and 384^2 with f = 3, the last
    through the radix-3 passes) at sampled probes against the FP64 PRISM oracle
    (tests/golden/config4_samples.json, written by make_config4_samples.py)."""
    import json
    eels = _gpu()
    from paper_1908_07628_amd.batch import Batch
    g = json.load(open(GOLD4))
    specs = synth.config4(n_specimens=64, workers=1)       # no fork from a GPU process
    torch.cuda.empty_cache()
    _say("config4 generated; fused batch of", len(specs))
    bf = Batch(specs, precision="fp16_split", n_streams=4, tuned=False, fused=True)
    bf.run_eager()
    bf.capture()
    bf.maps.zero_()
    torch.cuda.synchronize()
    bf.replay()
    maps = bf.maps_host()
    del bf
    torch.cuda.empty_cache()
    assert sorted(specs[s["index"]].nx for s in g["specimens"]) == [128, 256, 384]
    for s in g["specimens"]:
        got = maps[s["index"]][s["probe_index"]]
        ref = np.asarray(s["map"])
        _say("specimen", s["index"], "max rel err", float(np.max(np.abs(got - ref)) / np.max(ref)))
        assert np.all(np.isfinite(got)) and np.max(ref) > 0
        assert maps_close(got, ref, 1e-3)


def test_autotuner_caches_a_valid_setting(tmp_path, monkeypatch):
    eels = _gpu()
    from paper_1908_07628_amd import autotune
    monkeypatch.setenv("EELS_TUNE_CACHE", str(tmp_path / "tune.json"))
    p = _specimens(1, seed=11)[0]
    plan = eels.Plan(p, precision="bf16_split")
    V, H = eels.device_inputs(p)
    best, times = autotune.tune(plan, V, H, reps=1)
    pcs, lcs = autotune.plan_candidates(plan), autotune.candidates(plan)
    assert len(pcs) == 4 and len(times) == len(pcs) + len(lcs) - 1
    assert {k: best[k] for k in autotune.PLAN_KNOBS} in pcs
    assert {k: best[k] for k in autotune.KNOBS} in lcs
    assert autotune.load_cache()[autotune.key_of(plan)] == best
    assert autotune.plan_knobs(plan) == {k: best[k] for k in autotune.PLAN_KNOBS}
    assert autotune.apply(plan) == {k: best[k] for k in autotune.KNOBS}
    tp = autotune.tuned_plan(plan)
    ws = tp.alloc_workspace()
    out = torch.empty(tp.n_probes, dtype=torch.float64, device="cuda")
    tp.execute(V, H, out, ws)
    autotune.set_knobs(autotune.DEFAULTS)
    ref = prism.prism_map(p)
    assert maps_close(out.cpu().numpy(), ref, 1e-3)
    # every macro-tile shape gives the map to the same bar
    for pc in pcs:
        autotune.set_knobs(pc)
        q = plan.replan()
        autotune.set_knobs(autotune.PLAN_DEFAULTS)
        q.execute(V, H, out, q.alloc_workspace())
        assert maps_close(out.cpu().numpy(), ref, 1e-3), pc


@pytest.mark.parametrize("prec,detsum", [("fp32", "auto"), ("bf16_split", "auto"), ("bf16_split", "gram")])
def test_resident_s_matrices_serve_new_probes(prec, detsum):
    eels = _gpu()
    p = synth.config1()
    q = p.replace(probes=p.probes[:9] + [0.7, 0.4], probe_shape=(1, 9))
    a = eels.Plan(p, precision=prec, resident_s=True, detector_sum=detsum)
    b = eels.Plan(q, precision=prec, resident_s=True, detector_sum=detsum)
    assert a.s_signature() == b.s_signature()
    V, H = eels.device_inputs(p)
    ws = torch.empty(max(a.workspace_bytes, b.workspace_bytes), dtype=torch.uint8, device="cuda")
    outa = torch.empty(a.n_probes, dtype=torch.float64, device="cuda")
    outb = torch.empty(b.n_probes, dtype=torch.float64, device="cuda")
    a.execute(V, H, outa, ws)
    b.execute(V, H, outb, ws, flags=eels.EXEC_SKIP_SWEEPS)   # reuses the S-matrices of a
    torch.cuda.synchronize()
    ref = eels.solve(q, precision=prec, detector_sum=detsum)
    assert np.array_equal(outb.cpu().numpy(), ref)
    tol = 1e-4 if prec == "fp32" else 1e-3
    assert maps_close(outb.cpu().numpy(), prism.prism_map(q), tol)


def test_resident_s_matrices_serve_new_probes_window_gram():
    """Resident S-matrices reused for new probes (EXEC_SKIP_SWEEPS) in the window-Gram form
    (f = 2, cropped windows, the form forced): bitwise equal to a fresh solve of the new
    probes, and within the split bar of the oracle."""
    eels = _gpu()
    p = synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=5, f=2)
    q = p.replace(probes=p.probes + [0.31, -0.17])
    keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
        a = eels.Plan(p, precision="bf16_split", order="probe_first", resident_s=True)
        b = eels.Plan(q, precision="bf16_split", order="probe_first", resident_s=True)
        ref = eels.solve(q, precision="bf16_split", order="probe_first")
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
    assert a.s_signature() == b.s_signature()
    V, H = eels.device_inputs(p)
    ws = torch.empty(max(a.workspace_bytes, b.workspace_bytes), dtype=torch.uint8, device="cuda")
    outa = torch.empty(a.n_probes, dtype=torch.float64, device="cuda")
    outb = torch.empty(b.n_probes, dtype=torch.float64, device="cuda")
    a.execute(V, H, outa, ws)
    b.execute(V, H, outb, ws, flags=eels.EXEC_SKIP_SWEEPS)
    torch.cuda.synchronize()
    got = outb.cpu().numpy()
    assert np.array_equal(got, ref)
    assert maps_close(got, prism.prism_map(q), 1e-3)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_server_results_equal_alone_and_in_the_mix(prec, tol):
    """Requests served through eels_server_* (continuous batching on 3 streams) give maps bitwise
    equal to a lone solve of each problem, and within the precision's bar of the oracle.  The
    first request finishes before the rest arrive, so its repeat (new probes) runs on its
    resident S-matrices."""
    eels = _gpu()
    from paper_1908_07628_amd.serve import Server
    sp = _specimens(4, seed=13)
    reqs = [sp[1], sp[2], sp[0].replace(probes=sp[0].probes + 0.37), sp[3],
            sp[1].replace(probes=sp[1].probes + 0.11)]
    first = sp[0]
    solo = [eels.solve(r, precision=prec) for r in [first] + reqs]
    srv = Server(hbm_budget_bytes=int(40e9), max_slots=3, precision=prec)
    try:
        t0 = srv.submit(first)
        r0 = srv.wait(t0, timeout=300)
        assert r0.error is None and np.array_equal(r0.map, solo[0])
        tickets = [srv.submit(r) for r in reqs]
        res = [r0] + [srv.wait(t, timeout=300) for t in tickets]
        for k, r in enumerate(res):
            assert r.error is None, r.error
            assert np.array_equal(r.map, solo[k]), k
            assert maps_close(r.map, prism.prism_map(([first] + reqs)[k]), tol), k
        assert res[3].resident_hit                 # the repeat of the first specimen
        st = srv.latency_stats()
        _say("serve stats", st, srv.stats())
        assert st["n"] == len(res) and st["p99_s"] >= st["p50_s"] > 0
        assert srv.stats()["completed"] == len(res)
    finally:
        srv.close()


def test_server_evicts_and_readmits_under_a_small_budget():
    """A budget that holds one workspace: each new specimen evicts the idle resident one, a
    repeat of an evicted specimen runs afresh, a repeat of the resident one reuses it, and every
    map equals the lone solve."""
    eels = _gpu()
    from paper_1908_07628_amd.serve import Server
    sp = _specimens(2, seed=21)
    a, b = sp[0], sp[1]
    wa = eels.Plan(a, resident_s=True).workspace_bytes
    wb = eels.Plan(b, resident_s=True).workspace_bytes
    solo_a, solo_b = eels.solve(a), eels.solve(b)
    budget = max(wa, wb) + min(wa, wb) // 2          # either alone, never both
    srv = Server(hbm_budget_bytes=budget, max_slots=2)
    try:
        seq = [(a, solo_a, False), (b, solo_b, False), (a, solo_a, False), (a, solo_a, True)]
        for k, (p, ref, hit) in enumerate(seq):
            r = srv.wait(srv.submit(p), timeout=120)       # one at a time
            assert r.error is None and np.array_equal(r.map, ref), k
            assert r.resident_hit == hit, k
        st = srv.stats()
        _say("small-budget stats", st)
        assert st["evictions"] == 2 and st["resident_hits"] == 1 and st["resident_entries"] == 1
        assert st["resident_bytes"] <= budget
    finally:
        srv.close()


def test_server_rejects_request_over_budget():
    eels = _gpu()
    from paper_1908_07628_amd.serve import Server
    srv = Server(hbm_budget_bytes=int(1e6), max_slots=1, precision="fp32")
    try:
        with pytest.raises(eels.EelsError) as e:
            srv.submit(synth.config1())
        assert e.value.status == 5 and "budget" in str(e.value)      # EELS_ERR_OOM
    finally:
        srv.close()


def test_server_recovers_from_a_failed_request():
    """A request admitted under a budget larger than the device (the whole nanoparticle map with
    every slice's S-matrix data resident, about 2 TB) fails to allocate its workspace: it ends
    with EELS_ERR_OOM, and the slot and its footprint are released, so the next request runs."""
    eels = _gpu()
    from paper_1908_07628_amd.serve import Server
    big = synth.config3()
    small = _specimens(1, seed=5)[0]
    ref = eels.solve(small)
    srv = Server(hbm_budget_bytes=int(8e12), max_slots=1)
    try:
        r = srv.wait(srv.submit(big), timeout=120)
        _say("big request", r.status, r.error, r.workspace_bytes / 1e12, "TB")
        assert r.done and r.status == 5 and r.map is None
        st = srv.stats()
        assert st["failed"] == 1 and st["running_bytes"] == 0
        r2 = srv.wait(srv.submit(small), timeout=120)
        assert r2.error is None and np.array_equal(r2.map, ref)
    finally:
        srv.close()
