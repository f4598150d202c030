"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP32 path rel-L2 <= 1e-4 on the map, split-precision <= 1e-3 (the relative
L2 norm of Eq. nrmsse as read).  Component checks (FFT sweeps, GEMM) use bounds
derived from single-precision round-off of the operation.
"""
import sys

import numpy as np
import pytest

from maptol import maps_close
import synth
from oracle import conventional, metrics, prism
from oracle.common import make_setup

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_07628_amd import eels
    return eels


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ------------------------------------------------------------------ complex GEMM

@pytest.mark.parametrize("prec,tol", [("fp32", 2e-6), ("bf16_split", 3e-5), ("fp16_split", 3e-6)])
@pytest.mark.parametrize("m,n,k", [(64, 32, 16), (150, 200, 37), (257, 129, 300)])
def test_cgemm_against_float64(prec, tol, m, n, k):
    eels = _need_gpu()
    _say("cgemm", prec, m, n, k)
    rng = np.random.default_rng(m * 1000 + n + k)
    A = (rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))).astype(np.complex64)
    B = (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))).astype(np.complex64)
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C = eels.cgemm(dA, dB, prec).cpu().numpy()
    err = np.linalg.norm(C - ref) / np.linalg.norm(ref)
    assert err < tol, err
    nrm = eels.cgemm(dA, dB, prec, norm2=True).cpu().numpy()
    ref_n = (np.abs(ref) ** 2).sum(axis=0)
    assert np.max(np.abs(nrm - ref_n) / ref_n) < 10 * tol


@pytest.mark.parametrize("stages", [2, 3, 4, 5])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_cgemm_split_pipelines_agree(stages, order):
    """Every LDS pipeline variant and tile order of the split GEMM gives the same product
    (same accumulation order along k), and it matches FP64 within the split tolerance."""
    eels = _need_gpu()
    _say("cgemm pipeline", stages, order)
    m, n, k = 300, 270, 203            # several tiles, ragged in every dimension
    rng = np.random.default_rng(7)
    A = (rng.standard_normal((m, k)) + 1j * rng.standard_normal((m, k))).astype(np.complex64)
    B = (rng.standard_normal((n, k)) + 1j * rng.standard_normal((n, k))).astype(np.complex64)
    ref = A.astype(np.complex128) @ B.astype(np.complex128).T
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    s0, o0 = eels.tune_get(eels.TUNE_SC_STAGES), eels.tune_get(eels.TUNE_TILE_ORDER)
    try:
        eels.tune_set(eels.TUNE_SC_STAGES, 2)
        eels.tune_set(eels.TUNE_TILE_ORDER, 0)
        base = eels.cgemm(dA, dB, "bf16_split").cpu().numpy()
        base_n = eels.cgemm(dA, dB, "bf16_split", norm2=True).cpu().numpy()
        eels.tune_set(eels.TUNE_SC_STAGES, stages)
        eels.tune_set(eels.TUNE_TILE_ORDER, order)
        C = eels.cgemm(dA, dB, "bf16_split").cpu().numpy()
        nrm = eels.cgemm(dA, dB, "bf16_split", norm2=True).cpu().numpy()
    finally:
        eels.tune_set(eels.TUNE_SC_STAGES, s0)
        eels.tune_set(eels.TUNE_TILE_ORDER, o0)
    assert np.array_equal(C, base)
    assert np.array_equal(nrm, base_n)
    assert np.linalg.norm(C - ref) / np.linalg.norm(ref) < 3e-5


# ------------------------------------------------------------------ sweeps

def _small(seed=41, **kw):
    base = dict(n=64, ny=32, L=12.0, Ly=6.5, nz=4, n_sites=2, n_trans=2, det_inner_mrad=4.0,
                det_outer_mrad=22.0, aperture_mrad=18.0)
    base.update(kw)
    return synth.random_problem(seed, **base)


def test_s1_rows_match_oracle():
    eels = _need_gpu()
    p = _small()
    st = make_setup(p)
    plan = eels.Plan(p)
    V, H = eels.device_inputs(p)
    ws = plan.alloc_workspace()
    S1 = prism.forward_s1(p, st, range(p.n_slices))
    for j in range(p.n_slices):
        _say("S1 slice", j)
        g = plan.debug_s1(V, j, ws).cpu().numpy().astype(np.complex128) / (p.nx * p.ny)
        err = np.linalg.norm(g - S1[j]) / np.linalg.norm(S1[j])
        assert err < 2e-6 * (j + 1), (j, err)


def test_s2_rows_match_oracle():
    eels = _need_gpu()
    p = _small()
    st = make_setup(p)
    plan = eels.Plan(p)
    V, H = eels.device_inputs(p)
    ws = plan.alloc_workspace()
    for j, S2 in prism.reverse_s2(p, st, 0):
        _say("S2 slice", j)
        g = plan.debug_s2(V, j, ws).cpu().numpy().astype(np.complex128)
        err = np.linalg.norm(g - S2) / np.linalg.norm(S2)
        assert err < 2e-6 * (p.n_slices - j), (j, err)


@pytest.mark.parametrize("n", [16, 32, 128, 256, 384, 512, 1024])
def test_sweep_sizes(n):
    """Every compiled transform length (384 = 3 x 128: the radix-24/8/2 passes): one beam pair
    through two slices."""
    eels = _need_gpu()
    _say("sweep size", n)
    L = n * 0.1
    lam_mrad = 0.0196875e3
    p = synth.random_problem(50 + n, n=n, L=L, nz=2, n_sites=1, n_trans=1, aperture_mrad=lam_mrad * 2.2 / L,
                             det_outer_mrad=lam_mrad * 3.2 / L, atoms_per_slice=3)
    st = make_setup(p)
    plan = eels.Plan(p, real_space=(n == 384))      # the band basis needs power-of-two sides
    V, H = eels.device_inputs(p)
    ws = plan.alloc_workspace()
    S1 = prism.forward_s1(p, st, [1])[1]
    g = plan.debug_s1(V, 1, ws).cpu().numpy().astype(np.complex128) / (p.nx * p.ny)
    assert np.linalg.norm(g - S1) / np.linalg.norm(S1) < 1e-5
    for j, S2 in prism.reverse_s2(p, st, 0):
        if j == 0:
            g2 = plan.debug_s2(V, 0, ws).cpu().numpy().astype(np.complex128)
            assert np.linalg.norm(g2 - S2) / np.linalg.norm(S2) < 1e-5


# ------------------------------------------------------------------ whole maps

@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_radix3_grid_maps(prec, tol):
    """A 384 x 384 specimen (f = 3, 4 A crop, order P) of the batch workload's kind: the map
    through the radix-3 passes against the oracle; the full-cell band basis and the
    conventional multislice refuse the size."""
    eels = _need_gpu()
    rng = np.random.Generator(np.random.PCG64(384))
    p = synth.random_lattice_specimen(rng, 384, 3, 2, nt_range=(3, 3), det_outer_mrad=20.0, n_scan=8)
    assert p.nx == 384 and p.interp_f == 3
    ref = prism.prism_map(p)
    assert np.max(ref) > 0
    _say("384 grid", prec)
    got = _map(eels, p, prec)
    _say("  rel-L2", metrics.rel_l2(got, ref))
    assert maps_close(got, ref, tol)
    assert np.all(got[ref == 0] == 0)
    with pytest.raises(eels.EelsError):
        eels.Plan(p.replace(window_A=0.0, interp_f=1))



def _map(eels, p, precision="fp32", order="auto", **kw):
    return eels.solve(p, precision=precision, order=order, **kw)


def test_config1_fp32_matches_both_oracles():
    eels = _need_gpu()
    p = synth.config1()
    I1 = conventional.conventional_map(p)
    I2 = prism.prism_map(p)
    for order in ("auto", "s_first", "probe_first"):
        for real in (False, True):
            _say("config1", order, "real-space" if real else "band basis")
            g = _map(eels, p, "fp32", order, real_space=real)
            assert maps_close(g, I1, 1e-4)
            assert maps_close(g, I2, 1e-4)
            assert metrics.max_rel(g, I2) < 1e-4


@pytest.mark.parametrize("prec,tol", [("bf16_split", 1e-3), ("fp16_split", 1e-3)])
def test_config1_split_precision(prec, tol):
    eels = _need_gpu()
    p = synth.config1()
    I2 = prism.prism_map(p)
    for order in ("s_first", "probe_first"):
        for real in (False, True):
            _say("config1", prec, order, real)
            assert maps_close(_map(eels, p, prec, order, real_space=real), I2, tol)


CASES = {
    "nonsquare_annulus": dict(seed=61, n=64, ny=32, L=12.0, Ly=6.5, nz=4, n_sites=3, n_trans=3,
                              det_inner_mrad=4.0, det_outer_mrad=22.0, aperture_mrad=18.0),
    "crop_window": dict(seed=62, n=128, L=16.0, nz=5, n_sites=4, n_trans=2, window_A=3.0,
                        aperture_mrad=20.0, det_outer_mrad=30.0, n_scan=5),
    "crop_defocus": dict(seed=63, n=64, L=10.0, nz=3, n_sites=2, n_trans=3, window_A=4.0, defocus_A=25.0,
                         aperture_mrad=20.0, det_outer_mrad=28.0),
    "thin_and_thick": dict(seed=64, n=32, L=6.0, nz=7, n_sites=5, n_trans=1, dz=[1, 2, 3, 1.5, 2, 2.5, 1],
                           aperture_mrad=15.0, det_outer_mrad=20.0),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("order", ["s_first", "probe_first"])
@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_random_cases(name, order, prec, tol):
    eels = _need_gpu()
    kw = dict(CASES[name])
    p = synth.random_problem(kw.pop("seed"), **kw)
    _say("case", name, order, prec)
    ref = prism.prism_map(p)
    g = _map(eels, p, prec, order)
    assert maps_close(g, ref, tol)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3), ("fp16_split", 1e-3)])
def test_gram_detector_sum(prec, tol):
    """Gram form of the detector sum against the oracle and against the direct sum.  Config 1
    has N_1 = 325: three 128-row tiles with a ragged last one, so the lower tiles of G come
    from the conjugate transposes of upper ones."""
    eels = _need_gpu()
    p = synth.config1()
    ref = prism.prism_map(p)
    for real in ((False, True) if prec != "fp32" else (False,)):
        _say("gram", prec, "real-space" if real else "band basis")
        plan = eels.Plan(p, precision=prec, order="s_first", real_space=real, detector_sum="gram")
        assert plan.info()["gram_form"] == 1
        g = _map(eels, p, prec, "s_first", real_space=real, detector_sum="gram")
        d = _map(eels, p, prec, "s_first", real_space=real, detector_sum="direct")
        assert maps_close(g, ref, tol)
        assert metrics.rel_l2(g, d) < tol


def test_gram_detector_sum_many_sites_and_batches():
    """Several sites in several slices, cropped windows (split precision), and a memory budget
    that splits the contraction into more batches: same map within FP64 reduction order."""
    eels = _need_gpu()
    p = synth.random_problem(72, n=64, L=12.0, nz=6, n_sites=6, n_trans=3, window_A=3.0, atoms_per_slice=3,
                             aperture_mrad=18.0, det_outer_mrad=30.0)
    ref = prism.prism_map(p)
    full = eels.Plan(p, precision="bf16_split", detector_sum="gram")
    ws = full.info()["workspace_bytes"]
    small = eels.Plan(p, precision="bf16_split", detector_sum="gram", max_workspace_bytes=int(ws * 0.96))
    assert small.info()["n_batches"] > full.info()["n_batches"] or small.info()["n_groups"] > 1
    a = _map(eels, p, "bf16_split", detector_sum="gram")
    b = _map(eels, p, "bf16_split", detector_sum="gram", max_workspace_bytes=int(ws * 0.96))
    assert metrics.rel_l2(a, ref) < 1e-3
    assert metrics.rel_l2(a, b) < 1e-10


@pytest.mark.parametrize("prec", ["fp32", "bf16_split"])
def test_gram_stacked_rows_match_per_transition(prec):
    """The Gram form's first GEMM with the transitions' rows stacked into one problem (the
    default) and with one problem per transition computes every output element with the
    same accumulation order: the maps are bitwise equal.  Config 1: 3 transitions of 325
    rows, 975 stacked rows in 8 tiles instead of 3 x 3."""
    eels = _need_gpu()
    p = synth.config1()
    maps = []
    try:
        for stack in (1, 0):
            eels.tune_set(eels.TUNE_GRAM_STACK, stack)
            _say("gram stack", stack, prec)
            maps.append(_map(eels, p, prec, "s_first", detector_sum="gram"))
    finally:
        eels.tune_set(eels.TUNE_GRAM_STACK, 1)
    assert np.array_equal(maps[0], maps[1])
    assert maps_close(maps[0], prism.prism_map(p), (1e-4 if prec == "fp32" else 1e-3))


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
@pytest.mark.parametrize("detsum", ["gram", "direct"])
def test_gemm1_tile_rows_match(prec, detsum):
    """The split first GEMM with 256-row tiles (8 waves, the default) and with 128-row tiles
    accumulates every output element in the same order: bitwise-equal maps.  Config 1 (Gram:
    975 stacked rows, 4 tiles of 256 with a ragged last one; direct: M = N_2 = 1305) and a
    random cell with a crop window (real-space K)."""
    eels = _need_gpu()
    cases = [synth.config1(),
             synth.random_problem(77, n=64, L=12.0, nz=4, n_sites=3, n_trans=3, window_A=3.0, atoms_per_slice=3)]
    for p in cases:
        maps = []
        try:
            for rows in (1, 0):
                eels.tune_set(eels.TUNE_GEMM1_ROWS, rows)
                _say("gemm1 rows", rows, prec, detsum)
                maps.append(_map(eels, p, prec, "s_first", detector_sum=detsum))
        finally:
            eels.tune_set(eels.TUNE_GEMM1_ROWS, 1)
        assert np.array_equal(maps[0], maps[1])
        assert maps_close(maps[0], prism.prism_map(p), 1e-3)


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_order_p_split_tile_rows(prec):
    """Order P in split precision (the first product reads SC transposes of the S_1
    windows and gathers the eligible probes' rows of C).  256- and 128-row tiles of the first
    GEMM accumulate every element in the same order (bitwise-equal maps); 256- and 128-row
    tiles of the second GEMM group the FP32 partial sums differently (equal to 1e-6).  Both
    meet the split bar against the oracle.  Config 1 forced to order P in the band basis and
    in real space (where H multiplies the S_2 windows and Psi is the shared operand), and the
    f = 2 cell with crop windows (the same real-space form)."""
    eels = _need_gpu()
    c1 = synth.config1()
    for p, kw in ((c1, {}), (c1, dict(real_space=True)),
                  (synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=6, f=2), {})):
        ref = prism.prism_map(p)
        maps = {}
        try:
            for r1, r2 in ((1, 1), (0, 1), (1, 0)):
                eels.tune_set(eels.TUNE_GEMM1_ROWS, r1)
                eels.tune_set(eels.TUNE_GEMM2_ROWS, r2)
                _say("order P rows", r1, r2, prec, p.name, kw)
                maps[(r1, r2)] = _map(eels, p, prec, "probe_first", **kw)
        finally:
            eels.tune_set(eels.TUNE_GEMM1_ROWS, 1)
            eels.tune_set(eels.TUNE_GEMM2_ROWS, 1)
        assert np.array_equal(maps[(1, 1)], maps[(0, 1)])
        assert np.max(np.abs(maps[(1, 1)] - maps[(1, 0)])) <= 1e-6 * np.max(maps[(1, 0)])
        for m in maps.values():
            assert maps_close(m, ref, 1e-3)


def test_interpolation_factor_case():
    eels = _need_gpu()
    p = synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=6, f=2)
    ref = prism.prism_map(p)
    assert np.count_nonzero(ref) > 0
    for prec, tol in (("fp32", 1e-4), ("bf16_split", 1e-3)):
        for order in ("s_first", "probe_first"):
            _say("f=2", prec, order)
            assert maps_close(_map(eels, p, prec, order), ref, tol)


@pytest.mark.parametrize("f", [2, 4])
def test_interpolation_on_a_tiled_specimen(f):
    """f x f copies of a 32^2 cell with f = 2 and 4 (the nanoparticle's factor): the map against
    the oracle on the big cell, and against the small cell's conventional map times
    f^2 N_1 / N_1(f = 1) at probes that see a copy; probes that see none are exactly zero."""
    eels = _need_gpu()
    ps = synth.random_problem(41, n=32, L=8.0, nz=3, n_sites=1, n_trans=3, window_A=4.0,
                              aperture_mrad=15.0, det_outer_mrad=20.0)
    copies = np.array([ps.site_xy[0] + [i * ps.lx, j * ps.ly] for j in range(f) for i in range(f)])
    rng = np.random.default_rng(5)
    near = np.concatenate([c + rng.uniform(-1.5, 1.5, (5, 2)) for c in copies])
    far = copies + [ps.lx / 2, ps.ly / 2]
    pb = synth.tiled_problem(ps, f, np.concatenate([near, far]))
    ref = prism.prism_map(pb)
    small = conventional.conventional_map(ps.replace(probes=np.mod(pb.probes, [ps.lx, ps.ly]),
                                                     probe_shape=(1, pb.n_probes)))
    st = make_setup(pb)
    ratio = f * f * st.ab1.shape[0] / st.n1_fine
    n = len(near)
    for prec, tol in (("fp32", 1e-4), ("bf16_split", 1e-3)):
        for order in ("s_first", "probe_first"):
            _say("tiled f =", f, prec, order)
            got = _map(eels, pb, prec, order)
            assert maps_close(got, ref, tol)
            assert metrics.rel_l2(got[:n], ratio * small[:n]) < tol
            assert np.all(got[n:] == 0.0)


@pytest.mark.parametrize("prec,tol", [("bf16_split", 1e-3), ("fp16_split", 1e-3), ("fp32", 1e-4)])
def test_window_gram_form(prec, tol):
    """Order P with cropped windows in the window-Gram form (knob 6 = 2, forced on these
    few-probe cells, where the default picks the per-transition form): per site one Gram GEMM
    of the S_2 window, G = M o sum_t conj(H_t) H_t^T, and Re(Psi^H G Psi) per probe.  Against
    the oracle at the precision's bar (FP32 1e-4, split 1e-3) and against the per-transition
    products (f = 1, 2, 4)."""
    eels = _need_gpu()
    ps = synth.random_problem(41, n=32, L=8.0, nz=3, n_sites=1, n_trans=3, window_A=4.0,
                              aperture_mrad=15.0, det_outer_mrad=20.0)
    rng = np.random.default_rng(6)
    cases = [("nanoparticle-like f=2", synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=6, f=2)),
             ("random f=1 crop", synth.random_problem(12, n=64, L=12.0, nz=3, window_A=4.0, n_sites=3)),
             ("tiled f=4", synth.tiled_problem(ps, 4, rng.uniform(0.0, 32.0, (40, 2))))]
    for name, p in cases:
        ref = prism.prism_map(p)
        assert np.max(ref) > 0
        keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
        try:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)     # wherever it applies
            _say("window Gram", name, prec)
            got = _map(eels, p, prec, "probe_first")
            eels.tune_set(eels.TUNE_WINDOW_GRAM, 0)
            direct = _map(eels, p, prec, "probe_first")
        finally:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
        _say("  rel-L2 vs oracle", metrics.rel_l2(got, ref), "vs direct", metrics.rel_l2(got, direct))
        assert np.all(np.isfinite(got))
        assert metrics.rel_l2(got, ref) < tol
        assert np.max(np.abs(got - ref)) <= tol * np.max(ref)
        assert metrics.rel_l2(got, direct) < tol
        assert np.all(got[ref == 0] == 0)


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_window_gram_g_epilogue_matches_combine(prec):
    """Split window-Gram form: G formed in the Gram GEMM's epilogue (tuning key 9 = 1, the
    default) on 256-row tiles (key 10 = 1) and on 128-row tiles (the default), against the Gram
    tiles M and the separate combine pass (key 9 = 0).  All round G from the same FP32 M and S,
    in different orders, so the maps agree to FP32 rounding, and they meet the oracle; with and
    without the raster form, at 1, 3 and 9 transitions."""
    eels = _need_gpu()
    cases = [("nanoparticle-like f=2 raster", synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2), 2),
             ("random f=1 crop, 3 transitions", synth.random_problem(12, n=64, L=12.0, nz=3, window_A=4.0,
                                                                     n_sites=3, n_trans=3), 0),
             ("random f=1 crop, 1 transition", synth.random_problem(13, n=64, L=12.0, nz=3, window_A=4.0,
                                                                    n_sites=4, n_trans=1), 0)]
    keys = (eels.TUNE_WINDOW_GRAM, eels.TUNE_RASTER, eels.TUNE_WG_FUSED, eels.TUNE_GRAM_ROWS)
    keep = {k: eels.tune_get(k) for k in keys}
    try:
        for name, p, raster in cases:
            ref = prism.prism_map(p)
            eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
            eels.tune_set(eels.TUNE_RASTER, raster)
            maps = {}
            # (key 9, key 10): G epilogue on 256-row and on 128-row tiles, then the combine pass
            for fused, rows in ((1, 1), (1, 0), (0, 1)):
                eels.tune_set(eels.TUNE_WG_FUSED, fused)
                eels.tune_set(eels.TUNE_GRAM_ROWS, rows)
                _say("G epilogue", name, prec, "key 9 =", fused, "key 10 =", rows)
                maps[fused, rows] = _map(eels, p, prec, "probe_first")
            for k in ((1, 0), (0, 1)):
                _say("  ", k, "vs (1, 1)", metrics.rel_l2(maps[k], maps[1, 1]))
                assert metrics.rel_l2(maps[k], maps[1, 1]) < 1e-6
            _say("  vs oracle", metrics.rel_l2(maps[1, 1], ref))
            assert maps_close(maps[1, 1], ref, 1e-3)
            assert np.all(maps[1, 1][ref == 0] == 0)
    finally:
        for k, v in keep.items():
            eels.tune_set(k, v)


@pytest.mark.parametrize("prec,tol", [("bf16_split", 1e-3), ("fp16_split", 1e-3), ("fp32", 1e-4)])
def test_raster_form(prec, tol):
    """The raster form of the window-Gram detector sum (knob 7 = 2): Psi and G Psi for every
    probe of a raster aligned with the beam lattice by 64 x 64 DFTs over the beam lattice per
    window pixel.  Against the oracle at the precision's bar and against the window-Gram form
    without it (knob 7 = 0): a sparse raster (every 8th residue), a dense one (all 64 residues
    per axis, 4096 probes) and an f = 4 tiled specimen (its small cell's conventional map)."""
    eels = _need_gpu()
    ps = synth.random_problem(41, n=32, L=8.0, nz=3, n_sites=1, n_trans=3, window_A=4.0,
                              aperture_mrad=15.0, det_outer_mrad=20.0)
    g = np.arange(16) * 0.5                            # step L_small / 16 on the f = 4 tiled cell
    tiled_probes = np.stack(np.meshgrid(g + 0.25, g + 0.25, indexing="xy"), axis=-1).reshape(-1, 2)
    cases = [("f=2 sparse raster", synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2)),
             ("f=2 dense raster", synth.config3_subproblem(n=128, L=25.0, nz=3, n_scan=64, f=2)),
             ("f=4 tiled", synth.tiled_problem(ps, 4, tiled_probes))]
    for name, p in cases:
        ref = prism.prism_map(p)
        assert np.max(ref) > 0
        keep = (eels.tune_get(eels.TUNE_WINDOW_GRAM), eels.tune_get(eels.TUNE_RASTER))
        try:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)
            eels.tune_set(eels.TUNE_RASTER, 2)
            assert eels.Plan(p, precision=prec, order="probe_first").info()["raster_form"] == 64, name
            _say("raster form", name, prec, p.n_probes, "probes")
            got = _map(eels, p, prec, "probe_first")
            eels.tune_set(eels.TUNE_RASTER, 0)
            wg = _map(eels, p, prec, "probe_first")
        finally:
            eels.tune_set(eels.TUNE_WINDOW_GRAM, keep[0])
            eels.tune_set(eels.TUNE_RASTER, keep[1])
        _say("  rel-L2 vs oracle", metrics.rel_l2(got, ref), "vs window Gram", metrics.rel_l2(got, wg))
        assert maps_close(got, ref, tol)
        assert maps_close(got, wg, tol)
        assert np.all(got[ref == 0] == 0)


def test_window_gram_fp16_range_at_many_detector_beams():
    """N_2 = 8093 detector beams and 9 transitions: unscaled, the window Gram matrix's
    diagonal (about N_2 sum_t |H_t|^2, rows of S_2 of unit mean square) would reach about
    7e4 at a site's centre pixel, above the FP16 maximum 65504.  The FP16 window-Gram map
    (scaled by 2^-13) is finite and equals the BF16 per-transition map well within the
    split bar."""
    eels = _need_gpu()
    p = synth.random_problem(7, n=256, L=20.0, nz=3, n_sites=2, n_trans=9, window_A=4.0, aperture_mrad=20.0,
                             det_outer_mrad=50.0, n_scan=4)
    keep = eels.tune_get(eels.TUNE_WINDOW_GRAM)
    try:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 2)     # wherever it applies
        _say("window Gram FP16, N2 = 8093")
        wg = _map(eels, p, "fp16_split", "probe_first")
        eels.tune_set(eels.TUNE_WINDOW_GRAM, 0)
        direct = _map(eels, p, "bf16_split", "probe_first")
    finally:
        eels.tune_set(eels.TUNE_WINDOW_GRAM, keep)
    _say("  rel-L2 vs BF16 per-transition", metrics.rel_l2(wg, direct))
    assert np.all(np.isfinite(wg)) and np.max(direct) > 0
    assert metrics.rel_l2(wg, direct) < 1e-4


def test_repeat_is_bitwise_identical():
    eels = _need_gpu()
    p = synth.config1()
    a = _map(eels, p, "bf16_split")
    b = _map(eels, p, "bf16_split")
    assert np.array_equal(a, b)


def test_memory_budget_grouping_same_map():
    eels = _need_gpu()
    p = synth.random_problem(71, n=64, L=12.0, nz=8, n_sites=6, window_A=3.0, atoms_per_slice=3,
                             aperture_mrad=18.0, det_outer_mrad=30.0)
    full = eels.Plan(p)
    ws = full.info()["workspace_bytes"]
    small = eels.Plan(p, max_workspace_bytes=int(ws * 0.95))
    assert small.info()["n_groups"] > 1 or small.info()["n_batches"] > full.info()["n_batches"]
    a = _map(eels, p)
    b = _map(eels, p, max_workspace_bytes=int(ws * 0.95))
    assert metrics.rel_l2(a, b) < 1e-12
    assert metrics.rel_l2(a, prism.prism_map(p)) < 1e-4


def _checkpoint_budget(eels, p, prec):
    """A workspace budget at which the planner makes several slice groups without S_1
    checkpoints and at least one checkpoint when forced (tuning key 8 = 2); host planning only."""
    ws = eels.Plan(p, precision=prec).info()["workspace_bytes"]
    keep = eels.tune_get(eels.TUNE_CHECKPOINT)
    try:
        for frac in np.arange(0.99, 0.3, -0.01):
            b = int(ws * frac)
            try:
                eels.tune_set(eels.TUNE_CHECKPOINT, 0)
                a = eels.Plan(p, precision=prec, max_workspace_bytes=b).info()
                eels.tune_set(eels.TUNE_CHECKPOINT, 2)
                c = eels.Plan(p, precision=prec, max_workspace_bytes=b).info()
            except eels.EelsError:
                continue
            if a["n_groups"] > 1 and a["n_checkpoints"] == 0 and c["n_checkpoints"] > 0:
                return b
    finally:
        eels.tune_set(eels.TUNE_CHECKPOINT, keep)
    return None


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-3)])
def test_checkpointed_groups_same_map(prec, tol):
    """Slice groups that resume the forward sweep from saved S_1 states give the map of groups
    that sweep again from slice 0, bit for bit (the same kernels on the same states), and both
    meet the oracle."""
    eels = _need_gpu()
    p = synth.random_problem(82, n=64, L=12.0, nz=6, atoms_per_slice=20, n_sites=100, window_A=4.0,
                             aperture_mrad=18.0, det_outer_mrad=30.0)
    b = _checkpoint_budget(eels, p, prec)
    assert b is not None
    keep = eels.tune_get(eels.TUNE_CHECKPOINT)
    maps = {}
    try:
        for k in (0, 2):
            eels.tune_set(eels.TUNE_CHECKPOINT, k)
            _say("checkpoints", prec, "key 8 =", k, "budget", b)
            maps[k] = _map(eels, p, prec, max_workspace_bytes=b)
    finally:
        eels.tune_set(eels.TUNE_CHECKPOINT, keep)
    assert np.array_equal(maps[0], maps[2])
    assert maps_close(maps[2], prism.prism_map(p), tol)


def test_zero_transition_potential_gives_zero_map():
    eels = _need_gpu()
    p = synth.config1()
    g = _map(eels, p.replace(H=np.zeros_like(p.H)))
    assert np.all(g == 0)


def test_no_sites_gives_zero_map():
    eels = _need_gpu()
    p = synth.config1()
    q = p.replace(site_slice=p.site_slice[:0], site_xy=p.site_xy[:0], site_ntrans=p.site_ntrans[:0],
                  site_hoff=p.site_hoff[:0])
    assert np.all(_map(eels, q) == 0)


@pytest.mark.parametrize("prec", ["bf16_split", "fp16_split"])
def test_gemm_register_staging_same_maps(prec):
    """Tuning key 11 stages the split GEMMs' operands through registers instead of loading them
    straight into LDS (1: 256-row tiles, 2: all): the same tiles reach the same LDS positions, so every product (store, norm,
    Gram and G epilogues, 128- and 256-row tiles) and every map is bitwise the same."""
    eels = _need_gpu()
    cases = [("config1 order S", synth.config1(), "s_first", {}),
             ("crop order P per transition", synth.random_problem(12, n=64, L=12.0, nz=3, window_A=4.0,
                                                                  n_sites=3, n_trans=3), "probe_first",
              {eels.TUNE_WINDOW_GRAM: 0}),
             ("crop order P window Gram", synth.random_problem(13, n=64, L=12.0, nz=3, window_A=4.0,
                                                               n_sites=4, n_trans=2), "probe_first",
              {eels.TUNE_WINDOW_GRAM: 2, eels.TUNE_RASTER: 0}),
             ("raster 256-row Gram tiles", synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2),
              "probe_first", {eels.TUNE_WINDOW_GRAM: 2, eels.TUNE_RASTER: 2, eels.TUNE_GRAM_ROWS: 1}),
             ("raster, combine pass", synth.config3_subproblem(n=128, L=25.0, nz=5, n_scan=8, f=2),
              "probe_first", {eels.TUNE_WINDOW_GRAM: 2, eels.TUNE_RASTER: 2, eels.TUNE_WG_FUSED: 0})]
    keys = (eels.TUNE_WINDOW_GRAM, eels.TUNE_RASTER, eels.TUNE_GRAM_ROWS, eels.TUNE_WG_FUSED,
            eels.TUNE_GEMM_STAGING)
    keep = {k: eels.tune_get(k) for k in keys}
    try:
        for name, p, order, knobs in cases:
            for k, v in knobs.items():
                eels.tune_set(k, v)
            maps = []
            for staging in (0, 1, 2):
                eels.tune_set(eels.TUNE_GEMM_STAGING, staging)
                _say("register staging", name, prec, "key 11 =", staging)
                maps.append(_map(eels, p, prec, order))
            assert np.array_equal(maps[0], maps[1]) and np.array_equal(maps[0], maps[2]), name
            for k in knobs:
                eels.tune_set(k, keep[k])
        # the Gram form of order S (its Gram tiles in the SC kernel) and the debug GEMM
        p = synth.config1()
        maps = []
        for staging in (0, 2):
            eels.tune_set(eels.TUNE_GEMM_STAGING, staging)
            maps.append(eels.solve(p, precision=prec, order="s_first", detector_sum="gram"))
        assert np.array_equal(maps[0], maps[1])
    finally:
        for k, v in keep.items():
            eels.tune_set(k, v)
