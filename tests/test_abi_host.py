"""Host-side tests of the C ABI (no GPU needed): the library loads, exports every
function declared in include/eels.h, and plans problems exactly as the oracle does."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import physics as ph
from oracle.common import make_setup

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
eels = pytest.importorskip("paper_1908_07628_amd.eels")


def _lib():
    try:
        return eels.load_library()
    except ImportError as e:  # library not built
        pytest.skip(str(e))


def test_header_symbols_exported():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "eels.h")).read()
    names = set(re.findall(r"\b(eels_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(eels.EXPORTS) == names


def test_version_and_status_strings():
    lib = _lib()
    import ctypes as C
    a, b = C.c_int(), C.c_int()
    assert lib.eels_get_version(C.byref(a), C.byref(b)) == 0
    assert (a.value, b.value) == (0, 4)
    assert lib.eels_status_string(2) == b"beam outside the band limit"


@pytest.mark.parametrize("maker", [
    lambda: synth.config1(),
    lambda: synth.random_problem(3, n=32, ny=64, L=8.0, Ly=13.0, nz=3, det_inner_mrad=5.0),
    lambda: synth.random_problem(4, n=64, L=12.0, nz=3, window_A=3.0, interp_f=2, aperture_mrad=20.0,
                                 det_outer_mrad=25.0, n_scan=6),
])
def test_beam_lists_match_oracle(maker):
    _lib()
    p = maker()
    plan = eels.Plan(p)
    st = make_setup(p)
    assert np.array_equal(plan.beams(0), st.ab1)
    assert np.array_equal(plan.beams(1), st.ab2)
    inf = plan.info()
    assert inf["n_beams_in_fine"] == st.n1_fine
    assert inf["lambda_A"] == pytest.approx(st.lam, rel=1e-15)
    assert inf["sigma"] == pytest.approx(st.sigma, rel=1e-15)


def test_config_plan_shapes():
    _lib()
    inf = eels.Plan(synth.config1()).info()
    assert (inf["n_beams_in"], inf["n_beams_out"]) == (325, 1305)
    assert inf["n_live_x"] == 43 and inf["k_pixels"] == 64 * 64
    assert inf["order"] == eels.ORDER_PROBE_FIRST


def test_window_and_eligibility_match_oracle():
    _lib()
    p = synth.config3_subproblem()
    plan = eels.Plan(p)
    inf = plan.info()
    hx, hy = ph.window_geometry(p.nx, p.ny, p.lx, p.ly, p.window_A)
    assert (inf["window_nx"], inf["window_ny"]) == (2 * hx + 1, 2 * hy + 1)
    assert inf["k_pixels"] == (2 * hx + 1) * (2 * hy + 1)
    assert inf["k_stride"] % 16 == 0 and inf["k_stride"] >= inf["k_pixels"]


def test_plan_errors():
    _lib()
    p = synth.random_problem(1, n=32, L=8.0, nz=2)
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p.replace(det_outer_mrad=40.0))          # beyond the 26 mrad band
    assert e.value.status == 2
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p.replace(nx=48))                        # not a power of two
    assert e.value.status == 3
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p.replace(interp_f=2))                   # f > 1 needs a crop window
    assert e.value.status == 1
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p, max_workspace_bytes=1 << 20)          # budget below the fixed workspace
    assert e.value.status == 5
    bad = p.replace(site_slice=np.array([5, 0], dtype=np.int32))
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(bad)
    assert e.value.status == 1


def test_budget_splits_slices_into_groups():
    _lib()
    p = synth.random_problem(5, n=64, L=12.0, nz=8, n_sites=6, window_A=3.0, atoms_per_slice=3)
    full = eels.Plan(p).info()
    assert full["n_groups"] == 1
    ws = full["workspace_bytes"]
    small = eels.Plan(p, max_workspace_bytes=int(ws * 0.93)).info()
    assert small["workspace_bytes"] <= int(ws * 0.93)
    assert small["n_groups"] >= 2 or small["n_batches"] > full["n_batches"]


def test_checkpoints_cut_the_forward_sweeps_of_the_nanoparticle_map():
    """On the full nanoparticle workload at the bench's budget the S_1 windows need several
    slice groups; with S_1 checkpoints (tuning key 8 = 1, the default) the later groups resume
    from saved states, which the planner takes only where the sweeps then cost fewer passes."""
    _lib()
    p = synth.config3()
    budget = 296 * 10**9
    keep = eels.tune_get(eels.TUNE_CHECKPOINT)
    try:
        eels.tune_set(eels.TUNE_CHECKPOINT, 0)
        a = eels.Plan(p, precision="bf16_split", max_workspace_bytes=budget).info()
        eels.tune_set(eels.TUNE_CHECKPOINT, 1)
        b = eels.Plan(p, precision="bf16_split", max_workspace_bytes=budget).info()
    finally:
        eels.tune_set(eels.TUNE_CHECKPOINT, keep)
    assert a["n_groups"] > 1 and a["n_checkpoints"] == 0
    assert b["n_checkpoints"] >= 1 and b["workspace_bytes"] <= budget
    assert b["sweep_beam_slices"] < a["sweep_beam_slices"]
    # the transposed sweep runs once in both; the forward sweeps shrink
    n1, n2, nz = a["n_beams_in"], a["n_beams_out"], p.n_slices
    rev = n2 * (nz - int(np.min(p.site_slice)))
    assert (b["sweep_beam_slices"] - rev) / n1 < (a["sweep_beam_slices"] - rev) / n1
    with pytest.raises(eels.EelsError):
        eels.tune_set(eels.TUNE_CHECKPOINT, 3)
    with pytest.raises(eels.EelsError):
        eels.tune_set(eels.TUNE_WG_FUSED, 2)


def test_contraction_order_choice():
    _lib()
    p = synth.config1()
    a = eels.Plan(p, order="s_first").info()
    b = eels.Plan(p, order="probe_first").info()
    auto = eels.Plan(p).info()
    assert auto["gemm_flops"] == min(a["gemm_flops"], b["gemm_flops"])
    # order P for config 1: 8 (K N1 P + N2 Kc n_t P), Kc = band pixels (band basis) or K
    K, N1, N2, P, nt = 4096, 325, 1305, 16, 3
    Kb = b["band_pixels"]
    assert b["band_basis"] == 1 and 0.33 * K < Kb < 0.36 * K   # ~pi/9 of the grid
    assert b["gemm_flops"] == pytest.approx(8.0 * (K * N1 * P + N2 * Kb * nt * P))
    r = eels.Plan(p, order="probe_first", real_space=True).info()
    assert r["band_basis"] == 0
    assert r["gemm_flops"] == pytest.approx(8.0 * (K * N1 * P + N2 * K * nt * P))


def test_gram_detector_sum_plan():
    """Gram form: chosen automatically where it is cheaper (order S, f = 1), its flop count
    is the first product plus the Hermitian half of each site's Z^H Z plus one quadratic
    form per probe, and it is refused where it does not apply."""
    _lib()
    p = synth.config1()
    K, N1, N2, P, nt = 4096, 325, 1305, 16, 3
    d = eels.Plan(p, order="s_first", detector_sum="direct").info()
    g = eels.Plan(p, order="s_first", detector_sum="gram").info()
    assert d["gram_form"] == 0 and g["gram_form"] == 1
    Kb = g["band_pixels"]
    g1 = 8.0 * N2 * Kb * nt * N1
    assert d["gemm_flops"] == pytest.approx(g1 + 8.0 * nt * N2 * N1 * P)
    assert g["gemm_flops"] == pytest.approx(g1 + 8.0 * nt * N2 * N1 * (N1 + 1) / 2 + 8.0 * N1 * N1 * P)
    # 16 probes: the direct sum is cheaper, so auto keeps it
    assert eels.Plan(p, order="s_first").info()["gram_form"] == 0
    # many probes: auto switches to the Gram form
    many = p.replace(probes=np.tile(p.probes, (64, 1)), probe_shape=(32, 32))
    assert eels.Plan(many, order="s_first").info()["gram_form"] == 1
    assert eels.Plan(many, order="s_first", precision="bf16_split", real_space=True).info()["gram_form"] == 1
    for kw in (dict(order="probe_first"), dict(real_space=True)):          # FP32 real space: H in the prologue
        with pytest.raises(eels.EelsError) as e:
            eels.Plan(p, detector_sum="gram", **kw)
        assert e.value.status == 1
    f2 = synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=4, f=2)
    with pytest.raises(eels.EelsError):
        eels.Plan(f2, detector_sum="gram", precision="bf16_split")
    assert eels.Plan(f2, precision="bf16_split", order="s_first").info()["gram_form"] == 0


def test_image_detector_plan_rules():
    """Companion images: f = 1 only, at most EELS_MAX_IMAGES rings, inside the band limit."""
    _lib()
    p = synth.random_problem(3, n=64, L=9.0, nz=2, aperture_mrad=20.0, det_outer_mrad=30.0)
    ws0 = eels.Plan(p).info()["workspace_bytes"]
    ws1 = eels.Plan(p, images=[(0.0, 30.0), (35.0, 0.0)]).info()["workspace_bytes"]
    assert ws1 > ws0
    for bad, status in (([(0.0, 80.0)], 2),             # beyond the ~45 mrad band
                        ([(20.0, 10.0)], 1),            # outer below inner
                        ([(0.0, 5.0)] * 9, 1)):          # too many rings
        with pytest.raises(eels.EelsError) as e:
            eels.Plan(p, images=bad)
        assert e.value.status == status


def test_inverse_multislice_plan():
    """Inverse multislice: one slice's windows, a sweep to the exit and back, and no
    resident S-matrices."""
    _lib()
    p = synth.random_problem(6, n=64, L=10.0, nz=8, n_sites=6, atoms_per_slice=3, window_A=0.0)
    a = eels.Plan(p).info()
    b = eels.Plan(p, s1_mode="inverse").info()
    assert b["n_groups"] == 1 and b["workspace_bytes"] < a["workspace_bytes"]
    lowest = int(np.min(p.site_slice))
    assert b["sweep_beam_slices"] == (2 * p.n_slices - lowest) * b["n_beams_in"] + \
        (p.n_slices - lowest) * b["n_beams_out"]
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p, s1_mode="inverse", resident_s=True)
    assert e.value.status == 1


def test_s2_retreat_plan():
    """S_2 retreat: one slice's windows, S_2 to the entrance and back up to the top site beside
    S_1 up to it, real-space contraction, and no resident S-matrices."""
    _lib()
    p = synth.random_problem(6, n=64, L=10.0, nz=8, n_sites=6, atoms_per_slice=3, window_A=0.0)
    a = eels.Plan(p).info()
    b = eels.Plan(p, s1_mode="inverse_s2").info()
    assert a["band_basis"] == 1 and b["band_basis"] == 0
    assert b["n_groups"] == 1
    top = int(np.max(p.site_slice))
    assert b["sweep_beam_slices"] == (top + 1) * b["n_beams_in"] + (p.n_slices + top) * b["n_beams_out"]
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(p, s1_mode="inverse_s2", resident_s=True)
    assert e.value.status == 1
    with pytest.raises(KeyError):
        eels.Plan(p, s1_mode="retreat")


def test_band_table_matches_oracle_mask():
    """Band pixel count equals the oracle's circular mask count (same inclusive rule)."""
    _lib()
    from oracle import physics as ph
    for p in (synth.config1(), synth.random_problem(3, n=32, ny=64, L=8.0, Ly=13.0, nz=2)):
        inf = eels.Plan(p).info()
        assert inf["band_pixels"] == int(ph.band_mask(p.nx, p.ny, p.lx, p.ly).sum())


def test_conventional_entry_host_checks():
    """Conventional multislice: the workspace grows with the probe chunk by whole wave sets,
    and plans it cannot run (f > 1) or a missing workspace are refused before any device
    work."""
    import ctypes as C
    lib = _lib()
    p = synth.random_problem(4, n=32, nz=3, n_sites=2, n_trans=2)
    plan = eels.Plan(p)
    w1, w2, w3 = (plan.conventional_workspace_bytes(c) for c in (1, 2, 3))
    assert 0 < w1 < w2 < w3
    assert plan.conventional_workspace_bytes(0) == 0
    assert plan.conventional_chunk(w2) == 2 and plan.conventional_chunk(w2 - 1) == 1
    dummy = C.c_void_p(256)   # never dereferenced: the call fails its checks first
    st = lib.eels_conventional_map(plan._h, dummy, dummy, dummy, 2, None, 0, None)
    assert st == 4   # EELS_ERR_WORKSPACE
    q = synth.random_problem(4, n=64, L=16.0, nz=3, n_sites=2, n_trans=2, interp_f=2, window_A=3.0)
    plan2 = eels.Plan(q)
    st = lib.eels_conventional_map(plan2._h, dummy, dummy, dummy, 2, dummy, 1 << 40, None)
    assert st == 1   # EELS_ERR_INVALID_ARG
    assert "interp_f" in lib.eels_last_error().decode()


def test_tuning_knob_ranges_and_gram_stack_plan():
    """Knob values are range-checked; the Gram form's first GEMM stacks the transitions'
    rows by default (plan-time knob 3)."""
    _lib()
    for key, bad in ((0, 1), (0, 6), (1, 3), (2, 4), (3, 2), (3, -1), (4, 2), (5, 2), (5, -1), (6, 3), (6, -1),
                     (7, 3), (8, 3), (9, 2), (9, -1), (10, 2), (11, 3), (11, -1), (12, 0)):
        with pytest.raises(eels.EelsError):
            eels.tune_set(key, bad)
    assert eels.tune_get(eels.TUNE_GRAM_STACK) == 1 and eels.tune_get(eels.TUNE_GEMM1_ROWS) == 1
    assert eels.tune_get(eels.TUNE_GEMM2_ROWS) == 1 and eels.tune_get(eels.TUNE_WINDOW_GRAM) == 1
    assert eels.tune_get(eels.TUNE_CHECKPOINT) == 1 and eels.tune_get(eels.TUNE_WG_FUSED) == 1
    assert eels.tune_get(eels.TUNE_GRAM_ROWS) == 0 and eels.tune_get(eels.TUNE_GEMM_STAGING) == 1


def test_fused_batch_plan_checks():
    """Host side of the fused batch contraction: merged descriptors are built and bounds-
    checked against each plan's workspace region; mixed or FP32 precision, non-resident plans
    and overlapping or misaligned regions are refused."""
    _lib()
    probs = [synth.random_problem(40 + i, n=n, L=L, nz=3, n_sites=2, n_trans=2, window_A=w, interp_f=f)
             for i, (n, L, w, f) in enumerate([(32, 8.0, 0.0, 1), (64, 12.0, 3.0, 1), (64, 16.0, 3.0, 2),
                                                (32, 8.0, 3.0, 1)])]
    eels.tune_set(eels.TUNE_WINDOW_GRAM, 0)     # a fused batch takes the per-transition form
    try:
        _fused_batch_plan_checks(probs)
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 1)
    # the window-Gram form (order P, split, cropped windows; forced on this few-probe cell) is refused
    eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
    try:
        wg = [eels.Plan(probs[2], precision="bf16_split", order="probe_first", resident_s=True)]
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 1)
    with pytest.raises(eels.EelsError) as e:
        eels.FusedContraction(wg, [0], (wg[0].workspace_bytes + 255) // 256 * 256)
    assert e.value.status == 1 and "key 6" in str(e.value)


def _fused_batch_plan_checks(probs):
    for prec in ("bf16_split", "fp16_split"):
        plans = [eels.Plan(p, precision=prec, resident_s=True) for p in probs]
        sizes = [(pl.workspace_bytes + 255) // 256 * 256 for pl in plans]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        fc = eels.FusedContraction(plans, offs[:-1], int(offs[-1]))
        assert fc.table_bytes >= 144 * len(plans) * 2
        with pytest.raises(eels.EelsError) as e:                       # overlapping regions
            eels.FusedContraction(plans, [0] * len(plans), int(offs[-1]))
        assert e.value.status == 1
        with pytest.raises(eels.EelsError):                            # misaligned region
            eels.FusedContraction(plans, offs[:-1] + 8, int(offs[-1]) + 8)
        with pytest.raises(eels.EelsError):                            # beyond the arena
            eels.FusedContraction(plans, offs[:-1], int(offs[-1]) - 256)
    mixed = [eels.Plan(probs[0], precision="bf16_split", resident_s=True),
             eels.Plan(probs[1], precision="fp16_split", resident_s=True)]
    for bad in (mixed, [eels.Plan(probs[0], precision="fp32", resident_s=True)],
                [eels.Plan(probs[0], precision="bf16_split")]):
        sizes = [(pl.workspace_bytes + 255) // 256 * 256 for pl in bad]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        with pytest.raises(eels.EelsError) as e:
            eels.FusedContraction(bad, offs[:-1], int(offs[-1]))
        assert e.value.status == 1


def test_execute_flag_checks():
    """Execute flags are checked before any device work: unknown bits, SKIP_SWEEPS or
    SWEEPS_ONLY without resident S-matrices, both together, and SWEEPS_ONLY with companion
    images are refused."""
    import ctypes as C
    lib = _lib()
    p = synth.random_problem(5, n=32, nz=3, n_sites=2, n_trans=2)
    plain = eels.Plan(p, precision="bf16_split")
    res = eels.Plan(p, precision="bf16_split", resident_s=True)
    img = eels.Plan(p, precision="bf16_split", resident_s=True, images=[(0.0, 20.0)])
    dummy = C.c_void_p(256)   # never dereferenced: the calls fail their checks first
    ws = 1 << 40

    def run(plan, flags, images=None):
        return lib.eels_execute_images(plan._h, dummy, dummy, dummy, images, dummy, ws, None, flags)

    assert run(plain, 8) == 1
    assert run(plain, eels.EXEC_SKIP_SWEEPS) == 1
    assert run(plain, eels.EXEC_SWEEPS_ONLY) == 1
    assert run(res, eels.EXEC_SKIP_SWEEPS | eels.EXEC_SWEEPS_ONLY) == 1
    assert run(img, eels.EXEC_SWEEPS_ONLY, dummy) == 1
    assert "images" in lib.eels_last_error().decode()


def test_autotuner_plan_time_knobs(tmp_path, monkeypatch):
    """The tuner's macro-tile candidates (split precision only), the cache lookups, and the plan
    rebuilt with cached tile shapes, which leaves the global knobs at their defaults."""
    _lib()
    import json
    from paper_1908_07628_amd import autotune
    monkeypatch.setenv("EELS_TUNE_CACHE", str(tmp_path / "tune.json"))
    p = synth.config1()
    sp = eels.Plan(p, precision="bf16_split")
    fp = eels.Plan(p, precision="fp32")
    assert autotune.plan_candidates(fp) == [autotune.PLAN_DEFAULTS]
    pcs = autotune.plan_candidates(sp)
    assert len(pcs) == 4 and autotune.PLAN_DEFAULTS in pcs
    assert len({json.dumps(c, sort_keys=True) for c in pcs}) == 4
    assert autotune.plan_knobs(sp) == autotune.PLAN_DEFAULTS and autotune.tuned_plan(sp) is sp
    cfg = {"gemm1_rows": 0, "gemm2_rows": 1, "sc_stages": 3, "tile_order": 1}
    autotune.save_cache({autotune.key_of(sp): cfg})
    assert autotune.plan_knobs(sp) == {"gemm1_rows": 0, "gemm2_rows": 1}
    q = autotune.tuned_plan(sp)
    assert q is not sp and q.info() == sp.info() and q.workspace_bytes <= sp.workspace_bytes
    assert eels.tune_get(eels.TUNE_GEMM1_ROWS) == 1 and eels.tune_get(eels.TUNE_GEMM2_ROWS) == 1
    try:
        assert autotune.apply(sp) == {"sc_stages": 3, "tile_order": 1}
        assert eels.tune_get(eels.TUNE_SC_STAGES) == 3 and eels.tune_get(eels.TUNE_TILE_ORDER) == 1
    finally:
        autotune.set_knobs(autotune.DEFAULTS)


@pytest.mark.parametrize("precision", ["bf16_split", "fp32"])
def test_window_gram_form_chosen_by_flops(precision):
    """Order P with cropped windows, in split precision and in FP32: the default (knob 6 = 1)
    takes the window-Gram form where it needs fewer flops than the per-transition products
    (many eligible probes and transitions per site), and the per-transition form where few
    probes see each site; knob 2 forces the form and 0 turns it off.  The two forms lay out
    the contraction buffers differently, so the workspace size differs too."""
    _lib()

    def forms(p):
        out = {}
        try:
            for k in (0, 1, 2):
                eels.tune_set(eels.TUNE_WINDOW_GRAM, k)
                pl = eels.Plan(p, precision=precision, order="probe_first")
                out[k] = (pl.info()["window_gram_form"], pl.workspace_bytes)
        finally:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, 1)
        return out

    many = synth.random_problem(23, n=128, L=25.0, nz=3, n_sites=2, n_trans=9, window_A=4.0,
                                det_outer_mrad=25.0, n_scan=40)
    few = many.replace(probes=many.probes[:4], probe_shape=(1, 4))
    s = forms(many)
    assert [s[k][0] for k in (0, 1, 2)] == [0, 1, 1]
    assert s[1][1] == s[2][1] != s[0][1]
    s = forms(few)
    assert [s[k][0] for k in (0, 1, 2)] == [0, 0, 1]
    assert s[1][1] == s[0][1] != s[2][1]
    # full-cell windows and order S never take it
    full = many.replace(window_A=0.0)
    eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
    try:
        assert eels.Plan(full, precision=precision, order="probe_first").info()["window_gram_form"] == 0
        assert eels.Plan(many, precision=precision, order="s_first").info()["window_gram_form"] == 0
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 1)


def test_phase_names_match_the_header():
    """The binding's phase names are the header's EELS_PHASE_* in order (eels_timing_read
    fills one slot per phase)."""
    text = open(os.path.join(ROOT, "include", "eels.h")).read()
    ph = dict((m.group(1).lower(), int(m.group(2))) for m in re.finditer(r"EELS_PHASE_([A-Z0-9]+)\s*=\s*(\d+)", text))
    n = int(re.search(r"EELS_PHASES\s*=\s*(\d+)", text).group(1))
    assert len(eels.PHASES) == n == len(ph)
    for i, name in enumerate(eels.PHASES):
        assert ph[name] == i, name


def test_raster_form_needs_an_aligned_probe_raster():
    """The raster form of the window-Gram detector sum is taken only when every probe offset
    from the first is a whole multiple of L / (f M) (M = 64) in both axes and the aperture
    beams span fewer than M lattice columns and rows; knob 7 turns it off (0) or forces it (2),
    and the residues of the probes follow from the offsets."""
    _lib()
    keep = eels.tune_get(eels.TUNE_RASTER)
    try:
        p = synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=8, f=2)
        for prec in ("bf16_split", "fp32"):
            eels.tune_set(eels.TUNE_RASTER, 2)
            assert eels.Plan(p, precision=prec, order="probe_first").info()["raster_form"] == 64
            eels.tune_set(eels.TUNE_RASTER, 0)
            assert eels.Plan(p, precision=prec, order="probe_first").info()["raster_form"] == 0
        eels.tune_set(eels.TUNE_RASTER, 2)
        off = p.replace(probes=p.probes + np.array([0.37 * 25.0 / 128, 0.0]))     # a shared shift: still a raster
        assert eels.Plan(off, precision="fp32", order="probe_first").info()["raster_form"] == 64
        bent = p.probes.copy()
        bent[5, 0] += 0.01                                                        # one probe off the raster
        assert eels.Plan(p.replace(probes=bent), precision="fp32", order="probe_first").info()["raster_form"] == 0
        wide = synth.config3_subproblem(n=512, L=100.0, nz=3, n_scan=8, f=1)      # f = 1: a spans 203 columns
        assert eels.Plan(wide, precision="fp32", order="probe_first").info()["raster_form"] == 0
        full = p.replace(window_A=0.0, interp_f=1)
        assert eels.Plan(full, precision="fp32").info()["raster_form"] == 0
        with pytest.raises(eels.EelsError):
            eels.tune_set(eels.TUNE_RASTER, 3)
        # the nanoparticle map takes it by default
        eels.tune_set(eels.TUNE_RASTER, 1)
        big = synth.config3()
        assert eels.Plan(big, precision="bf16_split", max_workspace_bytes=int(290e9)).info()["raster_form"] == 64
    finally:
        eels.tune_set(eels.TUNE_RASTER, keep)


def test_grid_sides_384_with_crop_windows_only():
    """384 = 3 x 128 is a supported side for the sweeps (radix-3 passes) with cropped windows or
    the real-space contraction; the band basis needs powers of two; other sides are refused."""
    _lib()
    rng = np.random.Generator(np.random.PCG64(1))
    p = synth.random_lattice_specimen(rng, 384, 3, 2, nt_range=(3, 3), det_outer_mrad=20.0, n_scan=8)
    assert eels.Plan(p).info()["k_pixels"] > 0
    full = p.replace(window_A=0.0, interp_f=1)
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(full)
    assert e.value.status == 3
    assert eels.Plan(full, real_space=True).info()["band_basis"] == 0
    odd = synth.random_problem(3, n=48, L=8.0, nz=2)
    with pytest.raises(eels.EelsError) as e:
        eels.Plan(odd)
    assert e.value.status == 3
