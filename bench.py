"""EELS map throughput on one MI355X (probe positions per second).

Default workload: the nanoparticle map (1024 x 1024 px over 100 x 100 A, 50 slices of 2 A,
an 80 A bcc sphere of 22,659 atoms, every one ionised with 9 transitions, on a 20 A
amorphous support; PRISM interpolation factor f = 4, 4 A crop windows, 256 x 256 probes,
300 keV, 20 mrad aperture, 0-20 mrad detector).  A step is one complete map: set-up, both
scattering-matrix sweeps, every contraction and the FP64 reduction, with the inputs already
resident in HBM.

`value` is the BF16-split (hi+lo, FP32 accumulate) throughput.  The plain FP32 path runs
the same algorithm (window-Gram detector sum) and is timed on the whole map (`fp32`).
`roofline` is for the dominant kernel, timed with HIP events on the execute stream:
`achieved` counts the algorithmic complex-GEMM flops 8 M N K, `executed_frac` the three
MFMA products per multiply-add the split form runs.  `cpu_baseline` is the FP64 oracle
timed on a bounded sample of the same workload, on one core and on all host cores.

--steps and --warmup are upper bounds: the run stays inside --wall-budget seconds from
process start (the FP32 map and the CPU sample included) and reports the steps it timed.
Other workloads: --workload crystal | batch | serve.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "EELS map probe-px/s (FP32 plain vs BF16-split @1e-3 err); p50/p99 latency"
PEAK_BF16_TFLOPS = 2500.0
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0
WORKLOAD = ("perovskite crystal 256x256 px over 20x20 A, 50 slices x 2 A, 650 ionised B sites x 9 "
            "transitions (full-cell contraction), 64x64 probes, 300 keV, 21 mrad aperture, 0-50 mrad "
            "detector")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def subset_sites(p, keep):
    return p.replace(site_slice=p.site_slice[keep], site_xy=p.site_xy[keep],
                     site_ntrans=p.site_ntrans[keep], site_hoff=p.site_hoff[keep])


def gemm1_flops(info, p):
    """Useful complex flops of the first contraction GEMM (8 M N K summed over sites)."""
    kc = info["band_pixels"] if info["band_basis"] else info["k_pixels"]
    nt = float(np.sum(p.site_ntrans))
    return 8.0 * info["n_beams_out"] * kc * nt * info["n_beams_in"]


def cpu_baseline(p, budget_s=25.0):
    """FP64 conventional multislice (oracle) on one probe and the sites of the lowest ionised
    slice (their inelastic waves cross the most slices: about 12 s of CPU work); the time is
    scaled to the full site list with the per-probe multislice operation count
    n_z + sum_sites n_trans (n_z - j_site)."""
    from oracle import conventional
    ion = sorted(set(p.site_slice.tolist()))
    j = ion[0]
    keep = np.nonzero(p.site_slice == j)[0]
    q = subset_sites(p, keep).replace(probes=p.probes[:1], probe_shape=(1, 1))
    nz = p.n_slices
    ops_sample = nz + float(np.sum(q.site_ntrans * (nz - q.site_slice)))
    ops_full = nz + float(np.sum(p.site_ntrans * (nz - p.site_slice)))
    t0 = time.perf_counter()
    conventional.conventional_map(q, probe_chunk=1)
    dt = time.perf_counter() - t0
    per_probe = dt * ops_full / ops_sample
    return {
        "value": 1.0 / per_probe, "unit": "probe-px/s", "cores": 1, "kind": "oracle",
        "sample": (f"conventional multislice FP64 (numpy, one thread), 1 probe x {len(keep)} sites of "
                   f"ionised slice {j} ({dt:.1f} s); scaled by multislice operations "
                   f"{ops_full:.0f}/{ops_sample:.0f} to all {p.n_sites} sites"),
        "seconds_measured": round(dt, 2),
        "host_cpus": os.cpu_count(),
    }


def profile_sample(args):
    """Workload for hardware-counter runs: a plain 1 GiB device-to-device copy (known bytes,
    to calibrate FETCH_SIZE / WRITE_SIZE) and one map on the sites of the top N ionised
    slices of the crystal workload, whose contraction launches have the full map's shapes
    (nanoparticle workload: the sites of its N most populated ionised slices)."""
    import torch
    import synth
    from paper_1908_07628_amd import eels
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    budget = 0
    if args.workload == "nanoparticle":
        p = synth.config3()
        counts = np.bincount(p.site_slice, minlength=p.n_slices)
        top = np.argsort(-counts, kind="stable")[:args.profile_sample]
        q = subset_sites(p, np.nonzero(np.isin(p.site_slice, top))[0])
        free, _ = torch.cuda.mem_get_info()
        budget = int(free - (12 << 30))
    else:
        p = synth.config2()
        ion = sorted(set(p.site_slice.tolist()))
        q = subset_sites(p, np.nonzero(np.isin(p.site_slice, ion[-args.profile_sample:]))[0])
    V, H = eels.device_inputs(q)
    plan = eels.Plan(q, precision=args.precision, max_workspace_bytes=budget)
    ws = plan.alloc_workspace()
    out = torch.empty(q.n_probes, dtype=torch.float64, device="cuda")
    plan.execute(V, H, out, ws)
    torch.cuda.synchronize()
    print(json.dumps({"profile_sample": args.profile_sample, "sites": int(q.n_sites),
                      "copy_bytes": 2 * a.numel() * 4}), flush=True)


# sources whose change invalidates the committed counter figures of the contraction GEMMs (their
# kernels, the SC operand format, the descriptor and plan structures, and the planner that sets
# their shapes and batches)
TRAFFIC_SOURCES = ["kernels_gemm.hip", "sc_format.h", "internal.h", "plan.cpp"]


def sources_digest():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1908_07628_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def counter_values(name="k_cgemm_sc__config2_traffic_pmc.md"):
    """Calibrated HBM bytes from a committed counter summary under profiles/, if it was taken
    with the current kernel and planner sources (else an empty dict)."""
    summ = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(summ):
        return {}
    vals = {}
    for line in open(summ):
        if ":" in line and line.lstrip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("sources sha256") != sources_digest():
        return {}
    out = {}
    for k, v in vals.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def bench_batch(args):
    """Batching workload: 64 specimens of uneven size, one captured HIP graph."""
    import torch
    import synth
    from paper_1908_07628_amd import eels
    from paper_1908_07628_amd.batch import Batch
    t0 = time.time()
    specs = synth.config4(n_specimens=args.n_specimens, workers=min(16, os.cpu_count() or 1))
    log(f"{len(specs)} specimens generated in {time.time() - t0:.1f} s")
    b = Batch(specs, precision=args.precision, n_streams=4, tuned=False)
    log(f"arena {b.arena.numel() / 1e9:.1f} GB")
    t0 = time.time()
    b.tune(reps=1)
    log(f"autotuned in {time.time() - t0:.1f} s")
    # eager, one stream, one specimen after another (tables uploaded)
    b.tuned = False
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i, pl in enumerate(b.plans):
        V, H = b.inputs[i]
        pl.execute(V, H, b.out(i), b.workspaces[i])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    ref = b.maps_host()
    b.tuned = True
    b.capture()
    b.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        b.replay()
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t2) / args.steps
    got = b.maps_host()
    worst = max(float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300)) for g, r in zip(got, ref))
    probes = int(sum(p.n_probes for p in specs))
    arena_gb = b.arena.numel() / 1e9
    del b
    torch.cuda.empty_cache()
    # fused: the specimens' sweeps on the branches, then every level's GEMMs of all specimens
    # in one grouped launch (resident S-matrices; same tuned knobs for the sweeps)
    bf = Batch(specs, precision=args.precision, n_streams=4, tuned=True, fused=True)
    log(f"fused arena {bf.arena.numel() / 1e9:.1f} GB, merged table {bf.contraction.table_bytes} bytes")
    bf.run_eager()
    fused_eager = bf.maps_host()
    fused_vs = max(float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300)) for g, r in zip(fused_eager, ref))
    bf.capture()
    bf.replay()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(args.steps):
        bf.replay()
    torch.cuda.synchronize()
    t_fused = (time.perf_counter() - t3) / args.steps
    fused_graph = bf.maps_host()
    fused_stable = all(np.array_equal(g, r) for g, r in zip(fused_graph, fused_eager))
    del bf
    torch.cuda.empty_cache()
    # the same batch in plain FP32 (one captured graph on the same 4 branches)
    b32 = Batch(specs, precision="fp32", n_streams=4, tuned=False)
    b32.run_eager()
    m32 = b32.maps_host()
    b32.capture()
    b32.replay()
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(args.steps):
        b32.replay()
    torch.cuda.synchronize()
    t_fp32 = (time.perf_counter() - t4) / args.steps
    fp32_vs = max(float(np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-300)) for g, r in zip(ref, m32))
    del b32
    torch.cuda.empty_cache()
    return {
        "metric": METRIC, "value": round(probes / t_graph, 2), "unit": "probe-px/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": round(1e3 * t_graph, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.precision, "data": "synthetic",
        "config": {"workload": (f"batch of {len(specs)} specimens, grids {sorted(set(p.nx for p in specs))} "
                                "at 0.1 A/px, f = N/128, 10-80 slices, 1-20 ionised atoms x 3-9 transitions, "
                                "4 A crop, 16^2-64^2 probes; one captured HIP graph on 4 stream branches"),
                   "n_specimens": len(specs), "total_probes": probes},
        "eager_sequential_ms": round(1e3 * t_seq, 1), "graph_speedup": round(t_seq / t_graph, 2),
        "graph_vs_eager_max_rel_diff": worst, "arena_GB": round(arena_gb, 1),
        "fused": {"value": round(probes / t_fused, 2), "ms_per_step": round(1e3 * t_fused, 1),
                  "speedup_vs_graph": round(t_graph / t_fused, 3),
                  "max_rel_diff_vs_per_specimen": fused_vs, "graph_replays_equal_eager": fused_stable,
                  "what": ("specimens' sweeps on 4 stream branches, then each contraction level's GEMMs of "
                           "all specimens in one grouped launch per kernel variant (eels_batch_contract); "
                           "one captured graph")},
        "fp32": {"value": round(probes / t_fp32, 2), "ms_per_step": round(1e3 * t_fp32, 1),
                 "split_rel_l2_vs_fp32_worst": fp32_vs,
                 "what": "the same specimens in plain FP32, one captured graph on 4 stream branches"},
        "split_over_fp32": round(t_fp32 / t_graph, 2),
    }


def bench_serve(args):
    """Serving workload: Poisson arrivals, continuous batching, residency, p50/p99."""
    import torch
    import synth
    t0 = time.time()
    pool = synth.specimen_pool(55, args.pool, (128, 256, 512, 1024), (10, 60), (1, 20), (16, 64), "req",
                               workers=min(16, os.cpu_count() or 1))
    log(f"{len(pool)} specimens generated in {time.time() - t0:.1f} s")
    free, _ = torch.cuda.mem_get_info()
    out = {"metric": METRIC, "unit": "probe-px/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "dtype": args.precision, "vs_baseline": None,
           "config": {"workload": (f"Poisson stream of {args.n_requests} requests per rate over a pool of "
                                   f"{len(pool)} specimens (grids 128^2-1024^2, 10-60 slices), 30% repeats of "
                                   "(specimen, sites) with shifted probes; 4 slots"),
                      "budget_GB": round(0.8 * free / 1e9, 1)}, "rates": {}}
    precisions = args.serve_precisions or [args.precision]
    out["by_precision"] = {}
    for prec in precisions:
        out["rates"] = {}
        serve_rates(args, pool, free, prec, out)
        out["by_precision"][prec] = out["rates"]
    out["rates"] = out["by_precision"][precisions[0]]
    out["dtype"] = precisions[0]
    best = max(out["rates"].values(), key=lambda r: r["throughput_probe_px_s"])
    out["value"] = best["throughput_probe_px_s"]
    return out


def serve_rates(args, pool, free, precision, out):
    """One Poisson stream per rate through a fresh server (eels_server_*) in the given precision."""
    import synth
    from paper_1908_07628_amd.serve import Server
    for rate in args.rates:
        reqs = synth.config5_stream(seed=5, rate_per_s=rate, n_requests=args.n_requests, pool=pool)
        srv = Server(int(0.8 * free), max_slots=4, precision=precision)
        t0 = time.perf_counter()
        tickets = []
        for (t_arr, k, shift) in reqs:
            dt = t_arr - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            p = pool[k].replace(probes=pool[k].probes + shift)
            tickets.append(srv.submit(p))
        res = [srv.wait(t, timeout=900) for t in tickets]
        wall = time.perf_counter() - t0
        srv.close()
        st = srv.latency_stats(tickets)
        probes = sum(pool[k].n_probes for (_, k, _) in reqs)
        out["rates"][str(rate)] = {"p50_s": round(st["p50_s"], 3), "p99_s": round(st["p99_s"], 3),
                                   "mean_s": round(st["mean_s"], 3), "resident_hits": st["resident_hits"],
                                   "requests": st["n"], "errors": sum(r.error is not None for r in res),
                                   "throughput_probe_px_s": round(probes / wall, 1),
                                   "maps_per_s": round(len(reqs) / wall, 3)}
        log(f"{precision} rate {rate}: {out['rates'][str(rate)]}")


def serving_leg(args):
    """The metric's p50/p99 beside the map: one short Poisson stream (2 req/s, 24 requests,
    30% repeats with shifted probes) over 8 small seeded specimens through the eels_server_*
    loop in the bench precision.  A failure here is reported, not raised."""
    try:
        import torch
        import synth
        t0 = time.time()
        pool = synth.specimen_pool(57, 8, (128, 256, 512), (10, 40), (1, 20), (16, 64), "req",
                                   workers=min(16, os.cpu_count() or 1))
        free, _ = torch.cuda.mem_get_info()
        out = {"rates": {}}
        serve_rates(argparse.Namespace(rates=[2.0], n_requests=24), pool, free, args.precision, out)
        r = out["rates"]["2.0"]
        return {"workload": ("Poisson stream at 2 req/s, 24 requests over 8 seeded specimens (grids 128^2-512^2, "
                             "10-40 slices, 16^2-64^2 probes), 4 slots, S-matrices resident"),
                "precision": args.precision, "pool_s": round(time.time() - t0, 1), **r}
    except Exception as e:      # the map's line is printed either way
        return {"error": repr(e)}


NANO_WORKLOAD = ("nanoparticle 1024x1024 px over 100x100 A, 50 slices x 2 A: 80 A bcc sphere (22,659 atoms, "
                 "all ionised x 9 transitions) on a 20 A amorphous support (20,000 atoms); PRISM f = 4, 4 A crop "
                 "windows, 256x256 probes, 300 keV, 20 mrad aperture, 0-20 mrad detector")


_CPU = {}


def _oracle_sample(offset, sample_beams, sample_probes):
    """One bounded sample of the FP64 PRISM oracle on the nanoparticle workload (one BLAS
    thread): `sample_beams` aperture beams swept to the deepest ionised slice, as many detector
    beams swept from the exit to the shallowest (the oracle sweeps every beam this way), and one
    site's contraction (oracle.prism.contract_windows) on windows of the real shapes with
    `sample_probes` eligible probes.  Returns the seconds of each part."""
    import dataclasses
    import threadpoolctl
    from oracle import prism
    p, st, info = _CPU["p"], _CPU["st"], _CPU["info"]
    ion = sorted(set(p.site_slice.tolist()))
    with threadpoolctl.threadpool_limits(1):
        b = slice(offset, offset + sample_beams)
        st1 = dataclasses.replace(st, ab1=st.ab1[b], ix1=st.ix1[b], iy1=st.iy1[b], C=st.C[b])
        t0 = time.perf_counter()
        prism.forward_s1(p, st1, [ion[-1]])
        t_s1 = time.perf_counter() - t0
        st2 = dataclasses.replace(st, ab2=st.ab2[b], ix2=st.ix2[b], iy2=st.iy2[b])
        t0 = time.perf_counter()
        for _ in prism.reverse_s2(p, st2, j_stop=ion[0]):
            pass
        t_s2 = time.perf_counter() - t0
        rng = np.random.default_rng(offset)
        K, N1, N2 = info["k_pixels"], info["n_beams_in"], info["n_beams_out"]
        cplx = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
        S1w, S2w, C = cplx(N1, K), cplx(N2, K), cplx(N1, sample_probes)
        Hs = [cplx(K) for _ in range(int(p.site_ntrans[0]))]
        t0 = time.perf_counter()
        prism.contract_windows(S1w, S2w, C, Hs, 16.0)
        t_site = time.perf_counter() - t0
    return t_s1, t_s2, t_site


def cpu_baseline_nanoparticle(p, info, sample_beams=2, sample_probes=512, max_workers=16):
    """The FP64 PRISM oracle on a bounded sample of the nanoparticle map, scaled by operation
    counts to the whole map: N_1 / sample_beams x the S_1 sample + N_2 / sample_beams x the S_2
    sample + every site's contraction, which is linear in its eligible-probe count (mean over
    a seeded sample of sites).  Timed on one core, then with one process per core running the
    same sample on different beams at once (the beams and sites are independent, so the
    oracle parallelises this way); the all-core rate is the one-core rate times the work done
    per wall second."""
    import multiprocessing as mp
    from oracle.common import make_setup, site_eligible
    import threadpoolctl
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        st = make_setup(p.replace(probes=p.probes[:1], probe_shape=(1, 1)))
        t_setup = time.perf_counter() - t0
    _CPU.update(p=p, st=st, info=info)
    t_s1, t_s2, t_site = _oracle_sample(0, sample_beams, sample_probes)
    ion = sorted(set(p.site_slice.tolist()))
    pick = np.random.default_rng(1).choice(p.n_sites, size=min(64, p.n_sites), replace=False)
    # mean eligible-probe count per site on the full raster (the oracle's f > 1 rule)
    ps_mean = float(np.mean([np.sum(site_eligible(p, st, int(s))) for s in pick]))
    N1, N2 = info["n_beams_in"], info["n_beams_out"]
    one_core = t_setup + (N1 * t_s1 + N2 * t_s2) / sample_beams + p.n_sites * t_site * ps_mean / sample_probes
    sample_s = t_s1 + t_s2 + t_site
    n = max(1, min(max_workers, os.cpu_count() or 1))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(n) as pool:
        parts = pool.starmap(_oracle_sample, [(sample_beams * (k + 1), sample_beams, sample_probes) for k in range(n)])
    wall = time.perf_counter() - t0
    assert len(parts) == n
    speedup = n * sample_s / wall          # n samples' work per wall second, against one core
    all_core = one_core / speedup
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": p.n_probes / all_core, "unit": "probe-px/s", "cores": n, "kind": "oracle",
        "sample": (f"PRISM oracle FP64 (numpy FFT, one BLAS thread per process) on {n} processes, each sweeping "
                   f"{sample_beams} aperture beams to slice {ion[-1]} and {sample_beams} detector beams from the exit "
                   f"to slice {ion[0]} and contracting one site's windows with {sample_probes} probes "
                   f"({wall:.1f} s wall, {speedup:.1f}x the one-core rate); scaled to {N1} + {N2} beams and "
                   f"{p.n_sites} sites x {ps_mean:.0f} eligible probes (estimated {all_core / 3600:.1f} h per map)"),
        "one_core": {"value": p.n_probes / one_core, "cores": 1,
                     "sample": (f"set-up {t_setup:.1f} s, S_1 sample {t_s1:.1f} s, S_2 sample {t_s2:.1f} s, one "
                                f"site {t_site:.1f} s (estimated {one_core / 3600:.1f} h per map)")},
        "seconds_measured": round(t_setup + sample_s + wall, 1),
        "host_cpus": os.cpu_count(), "cpu_model": cpu_model,
    }


def check_against_oracle(maps, name="config3_map_samples.json"):
    """Errors of the GPU maps at the probes whose FP64 oracle values tests/golden holds (the
    whole map at 64 probes over the central 32 x 32; Eq. nrmsse read as relative L2, and the
    largest error over the largest sampled value)."""
    path = os.path.join(ROOT, "tests", "golden", name)
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    ref = np.asarray(g["map"])
    idx = np.asarray(g["probe_index"])
    out = {"probes": len(idx), "what": g["about"]}
    for k, m in maps.items():
        got = m[idx]
        out[k] = {"rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                  "max_err_over_max": float(np.max(np.abs(got - ref)) / np.max(ref))}
    return out


def bench_nanoparticle(args, t_proc0):
    """Nanoparticle workload: the f = 4, 4 A-crop map (order P, window-Gram detector sum) at
    full size, BF16 split timed over the steps, FP32 on one whole map."""
    import torch
    import synth
    from paper_1908_07628_amd import eels

    def elapsed():
        return time.time() - t_proc0

    t0 = time.time()
    p = synth.config3()
    log(f"inputs generated in {time.time() - t0:.1f} s: {p.n_sites} sites, {p.n_trans} transitions")
    V, H = eels.device_inputs(p)
    free, total = torch.cuda.mem_get_info()
    budget = int(free - (8 << 30))
    ion = sorted(set(p.site_slice.tolist()))

    # untimed kernel warm-up on the top ionised slice (loads the kernels; not a step)
    small = subset_sites(p, np.nonzero(p.site_slice == ion[-1])[0])
    for prec in (args.precision, "fp32"):
        wplan = eels.Plan(small, precision=prec, max_workspace_bytes=budget)
        wws = wplan.alloc_workspace()
        wout = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
        wplan.execute(V, H, wout, wws)
        torch.cuda.synchronize()
        del wws, wplan
    torch.cuda.empty_cache()

    plan = eels.Plan(p, precision=args.precision, max_workspace_bytes=budget)
    info = plan.info()
    ws = plan.alloc_workspace()
    out = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    log(f"plan: N1={info['n_beams_in']} N2={info['n_beams_out']} K={info['k_pixels']} "
        f"order={'S' if info['order'] == 1 else 'P'} window-Gram={info['window_gram_form']} "
        f"raster={info['raster_form']} "
        f"groups={info['n_groups']} batches={info['n_batches']} "
        f"workspace={info['workspace_bytes'] / 1e9:.1f} GB (budget {budget / 1e9:.0f} GB)")
    # warm-up steps: --warmup is an upper bound (a second one changes nothing measurable)
    n_warm, t_w = 0, None
    for w in range(max(1, min(args.warmup, 2))):
        t1 = time.perf_counter()
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        t_w = time.perf_counter() - t1
        n_warm += 1
        log(f"warmup step {w + 1} done ({t_w:.1f} s)")
    # steps: --steps is an upper bound; keep room for the FP32 map (about 3x a split step)
    # and the CPU sample inside the wall budget
    reserve = 3.5 * t_w + 20.0 + (0.0 if args.no_cpu_baseline else 75.0)
    fit = int((args.wall_budget - elapsed() - reserve) / t_w)
    steps = max(1, min(args.steps, fit))
    log(f"{elapsed():.0f} s since start; timing {steps} of at most {args.steps} steps")
    eels.timing_enable(1 << 16)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    phase_tot = {}
    for k in range(steps):
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        for name, v in eels.timing_read().items():
            a = phase_tot.setdefault(name, {"ms": 0.0, "count": 0})
            a["ms"] += v["ms"]
            a["count"] += v["count"]
        log(f"step {k + 1}/{steps} done")
    elapsed_steps = time.perf_counter() - t_start
    eels.timing_enable(0)
    value = p.n_probes * steps / elapsed_steps
    gpu_map = out.cpu().numpy()
    del ws
    torch.cuda.empty_cache()
    phases = {k: round(v["ms"] / steps, 1) for k, v in phase_tot.items()}

    # contraction kernels.  The plan's flop count is the per-transition form's,
    # sum over sites of 8 P_s K (N_1 + N_2 n_t), which gives the eligible probe-site pairs.
    # Per-transition form: the first product Psi = C S_1w (8 P_s K N_1 useful flops per site)
    # and the second A_n = (S_2w H_n) Psi (8 N_2 K n_t P_s).  Window-Gram form: the same first
    # product, the Gram GEMM M = S_2w^H S_2w (8 N_2 K (K + 1) / 2, the Hermitian half) and
    # G Psi (8 P_s K^2).  The roofline is that of the kernel with the most time.
    nt = set(p.site_ntrans.tolist())
    assert len(nt) == 1, "the flop split assumes one transition count"
    nt = float(nt.pop())
    N1, N2, K = info["n_beams_in"], info["n_beams_out"], info["k_pixels"]
    pairs = info["gemm_flops"] / (8.0 * K * (N1 + N2 * nt))
    split = args.precision != "fp32"

    raster = info.get("raster_form", 0) > 0

    def kernels(ph, wgram):
        if raster:
            # raster form: no first product; Z = G S_1w^T (8 K^2 N_1 per site), the Gram GEMM, and
            # the DFTs of Psi and Y over the beam lattice (VALU, timed as the raster phase)
            return {"gemm2": ("Z = G S_1w^T of the raster window-Gram form", 8.0 * K * K * N1 * p.n_sites,
                              "z_traffic_bytes_per_site"),
                    "gram": ("Gram GEMM M = S_2w^H S_2w of the window-Gram form (Hermitian half)",
                             8.0 * N2 * K * (K + 1) / 2.0 * p.n_sites, "gram_traffic_bytes_per_site")}
        k = {"gemm1": ("first product Psi = C S_1w", 8.0 * K * N1 * pairs, "gemm1_traffic_bytes_per_site")}
        if wgram:
            k["gemm2"] = ("G Psi product of the window-Gram form", 8.0 * K * K * pairs, "gpsi_traffic_bytes_per_site")
            k["gram"] = ("Gram GEMM M = S_2w^H S_2w of the window-Gram form (Hermitian half)",
                         8.0 * N2 * K * (K + 1) / 2.0 * p.n_sites, "gram_traffic_bytes_per_site")
        else:
            k["gemm2"] = ("second product (S_2w H_n) Psi", 8.0 * N2 * K * nt * pairs, "gemm2_traffic_bytes_per_site")
        return {name: v for name, v in k.items() if ph.get(name, {"count": 0})["count"] > 0}

    def contraction_table(ph, n_steps, prec):
        exec_factor = 3.0 if prec != "fp32" else 1.0
        peak = PEAK_BF16_TFLOPS if prec != "fp32" else PEAK_FP32_TFLOPS
        out_k = {}
        for name, (what, fl, _) in kernels(ph, ph.get("gram", {"count": 0})["count"] > 0).items():
            t = ph[name]
            useful = fl * n_steps / (t["ms"] * 1e-3) / 1e12
            out_k[name] = {"kernel": what, "ms": round(t["ms"] / n_steps, 1), "launches": t["count"] // n_steps,
                           "useful_complex_tflops": round(useful, 1), "frac": round(useful / peak, 4),
                           "executed_frac": round(exec_factor * useful / peak, 4)}
        return out_k

    wgram = phase_tot.get("gram", {"count": 0})["count"] > 0
    kern = kernels(phase_tot, wgram)
    contraction = contraction_table(phase_tot, steps, args.precision)
    dom = max(kern, key=lambda k: phase_tot[k]["ms"])
    what, dom_flops, ckey = kern[dom]
    g = phase_tot[dom]
    n_launch = g["count"] / steps
    avg_ms = g["ms"] / max(g["count"], 1)
    per_launch = dom_flops / n_launch
    exec_factor = 3.0 if split else 1.0
    peak = PEAK_BF16_TFLOPS if split else PEAK_FP32_TFLOPS
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    cv = counter_values("k_cgemm_sc__nanoparticle_traffic_pmc.md")
    traffic = cv[ckey] * p.n_sites / n_launch if ckey in cv else None
    roofline = {
        "bound": "mfma", "kernel": what + (" (k_cgemm_sc)" if split else " (k_cgemm)"),
        "achieved": round(achieved, 1), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
        "executed_frac": round(exec_factor * achieved / peak, 4),
        "traffic": traffic, "avg_launch_ms": round(avg_ms, 3), "launches_per_step": n_launch,
        "algorithmic_flops_per_launch": per_launch,
        "flop_definition": ("achieved: 8 M N K real flops per complex GEMM (the Gram GEMM: its Hermitian half); "
                            "executed_frac: the three BF16 MFMA products per complex multiply-add of the split "
                            "algorithm" if split else "8 M N K"),
    }
    nlx = info["n_live_x"]
    cap_bytes = 8.0 * p.n_sites * K * (N1 + N2)
    sweep_bytes = info["sweep_bytes"] + cap_bytes
    roofline_fft = {"sweeps": {
        "bound": "hbm", "kernels": "k_row_pass + k_col_pass (with S_1 and S_2 window captures)",
        "achieved": round(sweep_bytes / (phases["sweep"] * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
        "frac": round(sweep_bytes / (phases["sweep"] * 1e-3) / 1e9 / PEAK_HBM_GBPS, 4),
        "algorithmic_bytes_per_step": sweep_bytes,
        "byte_definition": (f"32 B x n_y x n_live_x ({nlx}) per beam-slice (2 passes, read + write; S_1 swept "
                            f"once per slice group) + 8 B per window pixel per beam captured")}}
    if raster and phases.get("raster", 0) > 0:
        # the DFTs of Psi and Y: two M^2-point 2-D FFTs per window pixel (5 N log2 N flops each),
        # reading the pixel's row of Xt and of Z (N_1 complex64 each)
        M2 = float(info["raster_form"]) ** 2
        fl = 2.0 * 5.0 * M2 * np.log2(M2) * K * p.n_sites
        by = 2.0 * 8.0 * N1 * K * p.n_sites
        t = phases["raster"] * 1e-3
        roofline_fft["raster_dft"] = {
            "bound": "alu", "kernels": "k_raster_dot", "achieved_tflops": round(fl / t / 1e12, 2),
            "peak_tflops": PEAK_FP32_TFLOPS, "frac": round(fl / t / 1e12 / PEAK_FP32_TFLOPS, 4),
            "achieved_GBps": round(by / t / 1e9, 1), "hbm_frac": round(by / t / 1e9 / PEAK_HBM_GBPS, 4),
            "definition": "2 x 5 M^2 log2(M^2) flops and 16 N_1 bytes read per window pixel per site"}

    # FP32: the same algorithm on the whole map, timed once
    fp32 = None
    m32 = None
    if not args.no_fp32:
        p32 = eels.Plan(p, precision="fp32", max_workspace_bytes=budget)
        i32 = p32.info()
        ws32 = p32.alloc_workspace()
        o32 = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
        log(f"FP32 plan: window-Gram={i32['window_gram_form']} groups={i32['n_groups']} "
            f"batches={i32['n_batches']} ({elapsed():.0f} s since start)")
        eels.timing_enable(1 << 16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p32.execute(V, H, o32, ws32)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t1
        ph32 = eels.timing_read()
        eels.timing_enable(0)
        del ws32
        torch.cuda.empty_cache()
        m32 = o32.cpu().numpy()
        fp32 = {"value": round(p.n_probes / dt32, 2), "ms_per_step": round(1e3 * dt32, 1), "steps": 1,
                "measured_on": "the whole map (same algorithm: order P, window-Gram detector sum" +
                               (", raster form)" if i32["raster_form"] else ")"),
                "window_gram_form": i32["window_gram_form"], "raster_form": i32["raster_form"],
                "phases_ms": {k: round(v["ms"], 1) for k, v in ph32.items() if v["count"]},
                "contraction_kernels": contraction_table(ph32, 1, "fp32"),
                "split_rel_l2_vs_fp32": float(np.linalg.norm(gpu_map - m32) / np.linalg.norm(m32))}
        log(f"FP32 map {dt32:.1f} s")

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "probe-px/s", "n_gpus": 1, "steps": steps,
        "warmup": n_warm, "ms_per_step": round(1e3 * elapsed_steps / steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if args.precision == "bf16_split" else args.precision,
        "data": "synthetic",
        "config": {"workload": NANO_WORKLOAD, "grid": [p.nx, p.ny], "n_slices": p.n_slices, "n_sites": p.n_sites,
                   "n_transitions": p.n_trans, "n_probes": p.n_probes, "N1": N1, "N2": N2, "window_pixels": K,
                   "interp_f": p.interp_f, "slice_groups": info["n_groups"], "batches": info["n_batches"],
                   "workspace_GB": round(info["workspace_bytes"] / 1e9, 1),
                   "precision": args.precision + " (hi+lo products, FP32 accumulate, FP64 map)"
                   if split else "fp32",
                   "contraction": "cropped windows, order P" + (", window-Gram detector sum" if wgram else "") +
                   (f", raster form (Psi and G Psi by {info['raster_form']}x{info['raster_form']} DFTs over the beam "
                    "lattice)" if raster else "")},
        "roofline": roofline, "contraction_kernels": contraction, "roofline_fft": roofline_fft,
        "phases_ms": phases, "fp32": fp32,
        "split_over_fp32": round(value / fp32["value"], 2) if fp32 else None,
        "map_sum": float(np.sum(gpu_map)),
    }
    maps = {args.precision: gpu_map}
    if m32 is not None:
        maps["fp32"] = m32
    result["check"] = check_against_oracle(maps)
    if not args.no_serve and elapsed() < args.wall_budget - 120:
        log(f"serving leg ({elapsed():.0f} s since start) ...")
        del V, H
        torch.cuda.empty_cache()
        result["serving"] = serving_leg(args)
    if not args.no_cpu_baseline:
        log(f"timing the CPU oracle sample ({elapsed():.0f} s since start) ...")
        result["cpu_baseline"] = cpu_baseline_nanoparticle(p, info)
    result["wall_s"] = round(elapsed(), 1)
    result["wall_budget_s"] = args.wall_budget
    return result


def main():
    t_proc0 = time.time()
    try:
        import psutil
        t_proc0 = psutil.Process().create_time()     # the wall budget counts from process start
    except Exception:
        pass
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="upper bound of the timed steps")
    ap.add_argument("--warmup", type=int, default=1, help="upper bound of the untimed warm-up steps")
    ap.add_argument("--wall-budget", type=float, default=450.0,
                    help="seconds from process start the run stays within (steps are cut to fit)")
    ap.add_argument("--precision", default="bf16_split", choices=["bf16_split", "fp16_split", "fp32"])
    ap.add_argument("--no-fp32", action="store_true", help="nanoparticle: skip the FP32 whole-map leg")
    ap.add_argument("--fp32-sample", action="store_true",
                    help="crystal: estimate FP32 from the top ionised slices instead of timing the whole map")
    ap.add_argument("--fp32-slices", type=int, default=2, help="ionised slices of the crystal FP32 sample and extras")
    ap.add_argument("--extras", action="store_true",
                    help="crystal: also time companion images, inverse multislice and conventional multislice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="nanoparticle: skip the short serving leg (p50/p99)")
    ap.add_argument("--check", action="store_true", help="crystal: compare sampled probes with the stored FP64 values")
    ap.add_argument("--workload", default="nanoparticle", choices=["nanoparticle", "crystal", "batch", "serve"],
                    help="nanoparticle: the f = 4 cropped-window map (default); crystal: the 256^2 full-cell map; "
                         "batch: 64 uneven specimens in one graph; serve: Poisson request stream with p50/p99 "
                         "latency")
    ap.add_argument("--profile-sample", type=int, default=0, metavar="N",
                    help="for counter runs: a 1 GiB device copy (calibration), then one map on the "
                         "top N ionised slices; prints one line")
    ap.add_argument("--conv-probes", type=int, default=32,
                    help="probes of the conventional-multislice comparison (0: skip)")
    ap.add_argument("--n-specimens", type=int, default=64)
    ap.add_argument("--pool", type=int, default=10)
    ap.add_argument("--n-requests", type=int, default=40)
    ap.add_argument("--rates", type=float, nargs="+", default=[1.0, 4.0])
    ap.add_argument("--serve-precisions", nargs="+", choices=["bf16_split", "fp16_split", "fp32"], default=None,
                    help="serving workload: run the request streams once per precision (default: --precision)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); this build runs on a "
              "single GPU and its multi-GPU layout (sites sharded over GPUs, one all-reduce of the map) "
              "is not run.", file=sys.stderr)
        sys.exit(2)
    if args.profile_sample > 0:
        profile_sample(args)
        return
    if args.precision == "bf16_split" and args.workload == "batch":
        args.precision = "fp16_split"
    fn = {"batch": lambda a, t: bench_batch(a), "serve": lambda a, t: bench_serve(a),
          "nanoparticle": bench_nanoparticle, "crystal": bench_crystal}[args.workload]
    print(json.dumps(fn(args, t_proc0)), flush=True)


def bench_crystal(args, t_proc0):
    """Crystal workload: the 256^2 full-cell map (band basis, order S, Gram detector sum)."""
    import torch
    import synth
    from paper_1908_07628_amd import eels

    t0 = time.time()
    p = synth.config2()
    log(f"inputs generated in {time.time() - t0:.1f} s: {p.n_sites} sites, {p.n_trans} transitions")
    V, H = eels.device_inputs(p)
    free, total = torch.cuda.mem_get_info()

    # untimed warm-up on one slice of the workload (loads the kernels; not a step)
    ion = sorted(set(p.site_slice.tolist()))
    small = subset_sites(p, np.nonzero(p.site_slice == ion[-1])[0])
    wplan = eels.Plan(small, precision=args.precision)
    wws = wplan.alloc_workspace()
    wout = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    wplan.execute(V, H, wout, wws)
    torch.cuda.synchronize()
    del wws, wplan

    plan = eels.Plan(p, precision=args.precision)
    info = plan.info()
    ws = plan.alloc_workspace()
    out = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    log(f"plan: N1={info['n_beams_in']} N2={info['n_beams_out']} band pixels={info['band_pixels']} "
        f"order={'S' if info['order'] == 1 else 'P'} batches={info['n_batches']} "
        f"workspace={info['workspace_bytes'] / 1e9:.1f} GB (free {free / 1e9:.0f} GB)")
    n_warm, t_w = 0, None
    for w in range(max(1, min(args.warmup, 2))):      # --warmup is an upper bound
        t1 = time.perf_counter()
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        t_w = time.perf_counter() - t1
        n_warm += 1
        log(f"warmup step {w + 1} done ({t_w:.1f} s)")
    # --steps is an upper bound: room for the FP32 map (about 4x a split step) and the CPU sample
    reserve = (0.5 if args.fp32_sample else 4.5) * t_w + 20.0 + (0.0 if args.no_cpu_baseline else 40.0)
    args.steps = max(1, min(args.steps, int((args.wall_budget - (time.time() - t_proc0) - reserve) / t_w)))
    args.warmup = n_warm
    log(f"timing {args.steps} steps")

    eels.timing_enable(8192)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    phase_tot = {}
    for k in range(args.steps):
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        ph = eels.timing_read()
        for name, v in ph.items():
            a = phase_tot.setdefault(name, {"ms": 0.0, "count": 0})
            a["ms"] += v["ms"]
            a["count"] += v["count"]
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    eels.timing_enable(0)
    ms_per_step = 1e3 * elapsed / args.steps
    value = p.n_probes * args.steps / elapsed
    gpu_map = out.cpu().numpy()

    counters = counter_values()
    # roofline of the dominant kernel (first contraction GEMM)
    g1 = phase_tot["gemm1"]
    g1_flops = gemm1_flops(info, p)
    n_launch_per_step = g1["count"] / args.steps
    avg_ms = g1["ms"] / max(g1["count"], 1)
    split = args.precision != "fp32"
    exec_factor = 3.0 if split else 1.0           # hi*hi + hi*lo + lo*hi
    per_launch = g1_flops / n_launch_per_step
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_BF16_TFLOPS if split else PEAK_FP32_TFLOPS
    roofline = {
        "bound": "mfma", "kernel": "k_cgemm_sc (first contraction GEMM)" if split else "k_cgemm",
        "achieved": round(achieved, 1), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
        "executed_frac": round(exec_factor * achieved / peak, 4),
        "traffic": counters.get("gemm1_traffic_bytes_per_launch") if split else None,
        "avg_launch_ms": round(avg_ms, 3),
        "launches_per_step": n_launch_per_step,
        "algorithmic_flops_per_launch": per_launch,
        "flop_definition": ("achieved: 8 M N K real flops per complex GEMM; executed_frac: the three BF16 MFMA "
                            "products per complex multiply-add of the split algorithm" if split else "8 M N K"),
    }
    phases = {k: round(v["ms"] / args.steps, 2) for k, v in phase_tot.items()}

    # HBM rooflines of the FFT passes: both sweeps (row + column passes with their window
    # and band captures) and the producer (band FFT of T H S_1 per site and transition)
    n_ion = info["n_ion_slices"]
    kwin = info["k_pixels"]
    cap_bytes = 8.0 * n_ion * (info["n_beams_in"] * kwin + info["n_beams_out"] * info["band_pixels"])
    sweep_bytes = info["sweep_bytes"] + cap_bytes
    sweep_s = phases["sweep"] * 1e-3
    nt_tot = float(np.sum(p.site_ntrans))
    prod_bytes = 8.0 * ((p.n_sites * info["n_beams_in"] + nt_tot) * kwin
                        + nt_tot * info["n_beams_in"] * info["band_pixels"])
    prod_s = phases["producer"] * 1e-3
    roofline_fft = {
        "sweeps": {"bound": "hbm", "kernels": "k_row_pass + k_col_pass (with S_1 window and S_2 band captures)",
                   "achieved": round(sweep_bytes / sweep_s / 1e9, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                   "frac": round(sweep_bytes / sweep_s / 1e9 / PEAK_HBM_GBPS, 4),
                   "traffic": ({"k_row_pass<256,1>": counters["row_pass_traffic_bytes_per_launch"],
                                "k_col_pass<256,1>": counters["col_pass_traffic_bytes_per_launch"],
                                "algorithmic_bytes_per_launch": 16.0 * info["n_beams_out"] * p.ny * info["n_live_x"]}
                               if "row_pass_traffic_bytes_per_launch" in counters else None),
                   "algorithmic_bytes_per_step": sweep_bytes,
                   "byte_definition": "32 B x n_y x n_live_x per beam-slice (2 passes, read + write) + captures"},
        "producer": {"bound": "hbm", "kernels": "k_band_rows + k_band_cols",
                     "achieved": round(prod_bytes / prod_s / 1e9, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                     "frac": round(prod_bytes / prod_s / 1e9 / PEAK_HBM_GBPS, 4), "traffic": None,
                     "algorithmic_bytes_per_step": prod_bytes,
                     "byte_definition": ("read S_1 windows and H once per site, write the band-basis operand; "
                                         "the row-to-column scratch round trip is not counted")},
    }

    del ws
    torch.cuda.empty_cache()
    companion = inverse = conv = None
    ps = subset_sites(p, np.nonzero(np.isin(p.site_slice, ion[-args.fp32_slices:]))[0])
    if args.extras:
        companion, inverse, conv = crystal_extras(args, p, ps, ion, V, H, info, value, gpu_map)
    return crystal_finish(args, t_proc0, p, ps, ion, V, H, info, value, gpu_map, elapsed, ms_per_step,
                          roofline, roofline_fft, phases, companion, inverse, conv)


def crystal_extras(args, p, ps, ion, V, H, info, value, gpu_map):
    """Companion images, the inverse-multislice S_1 and the conventional multislice on the GPU
    (--extras)."""
    import torch
    from paper_1908_07628_amd import eels
    # Extras, on the sites of the top ionised slices (their costs do not grow with the site
    # count except the contractions): companion images (iBF with the EELS detector's angles,
    # ADF from 60 mrad to the band limit) computed with the map, and the inverse-multislice
    # S_1 (Sec. 4.C) against the exact path.
    rings = [(p.det_inner_mrad, p.det_outer_mrad), (60.0, 0.0)]

    def timed(plan, with_images=False):
        wsx = plan.alloc_workspace()
        o = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
        im = torch.empty((max(plan.n_images, 1), p.n_probes), dtype=torch.float64, device="cuda")
        run = (lambda: plan.execute_images(V, H, o, im, wsx)) if with_images else (lambda: plan.execute(V, H, o, wsx))
        run()                                       # warm
        eels.timing_enable(8192)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        ph = eels.timing_read()
        eels.timing_enable(0)
        return dt, ph, o.cpu().numpy(), im.cpu().numpy(), plan.workspace_bytes

    base_plan = eels.Plan(ps, precision=args.precision)
    dt0, ph0, m0, _, ws0 = timed(base_plan)
    del base_plan
    dti, phi, mi, imgs, _ = timed(eels.Plan(ps, precision=args.precision, images=rings), with_images=True)
    companion = {
        "measured_on": f"sites of the top {args.fp32_slices} ionised slices",
        "rings_mrad": [[a, b if b > 0 else "band limit"] for a, b in rings],
        "images_phase_ms": round(phi["images"]["ms"], 2),
        "extra_sweep_ms": round(phi["sweep"]["ms"] - ph0["sweep"]["ms"], 2),
        "map_unchanged": bool(np.array_equal(mi, m0)),
        "ibf_mean": float(imgs[0].mean()), "adf_mean": float(imgs[1].mean()),
    }
    dtv, phv, mv, _, wsv = timed(eels.Plan(ps, precision=args.precision, s1_mode="inverse"))
    inverse = {
        "measured_on": f"sites of the top {args.fp32_slices} ionised slices",
        "map_rel_l2_vs_exact": float(np.linalg.norm(mv - m0) / np.linalg.norm(m0)),
        "ms_exact": round(1e3 * dt0, 1), "ms_inverse": round(1e3 * dtv, 1),
        "sweep_ms_exact": round(ph0["sweep"]["ms"], 1), "sweep_ms_inverse": round(phv["sweep"]["ms"], 1),
        "workspace_GB_exact": round(ws0 / 1e9, 2), "workspace_GB_inverse": round(wsv / 1e9, 2),
    }

    # Conventional multislice (Sec. 3, first algorithm) on the same GPU and the same specimen:
    # every transition's inelastic wave of every probe multisliced to the exit, on a block of
    # probes (its cost per probe does not depend on the probe)
    conv = None
    if args.conv_probes > 0:
        idx = np.arange(args.conv_probes) * (p.n_probes // args.conv_probes)
        q = p.replace(probes=p.probes[idx], probe_shape=(1, len(idx)))
        cplan = eels.Plan(q)
        torch.cuda.empty_cache()
        free_now, _ = torch.cuda.mem_get_info()
        chunk = min(len(idx), cplan.conventional_chunk(int(0.7 * free_now)))
        wsc = torch.empty(cplan.conventional_workspace_bytes(chunk), dtype=torch.uint8, device="cuda")
        oc = torch.empty(len(idx), dtype=torch.float64, device="cuda")
        eels.timing_enable(8192)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        cplan.conventional_map(V, H, oc, chunk, wsc)
        torch.cuda.synchronize()
        dtc = time.perf_counter() - t1
        phc = eels.timing_read()
        eels.timing_enable(0)
        del wsc
        mc = oc.cpu().numpy()
        # algorithmic HBM bytes: every row or column pass reads and writes one wave plane of
        # n_y x n_live_x complex64 (elastic: rows of slices 0..j_last, columns of 0..j_last-1;
        # a transition of slice s: columns of s..n_z-1, rows of s+1..n_z-1); the entrance wave
        # written once per ionised slice and read once per site; H read once per chunk; the
        # new waves written; the exit band coefficients written
        nlx = info["n_live_x"]
        plane = 8.0 * p.ny * nlx
        full = 8.0 * p.nx * p.ny
        n_c = len(idx)
        j_last = int(np.max(p.site_slice))
        nt_s = p.site_ntrans.astype(np.float64)
        passes = n_c * (2 * j_last + 1 + float(np.sum(nt_s * (2 * (p.n_slices - p.site_slice) - 1))))
        n_ion = len(set(p.site_slice.tolist()))
        spawn = n_c * (n_ion * full + p.n_sites * full + nt_s.sum() * plane) + \
            -(-n_c // chunk) * nt_s.sum() * full
        conv_bytes = 2.0 * plane * passes + spawn + n_c * nt_s.sum() * 8.0 * info["band_pixels"]
        conv_rate = len(idx) / dtc
        conv = {
            "measured_on": f"{len(idx)} probes of the raster, {chunk} at a time, all {p.n_sites} sites",
            "value": round(conv_rate, 3), "unit": "probe-px/s", "ms": round(1e3 * dtc, 1),
            "phases_ms": {k: round(v["ms"], 1) for k, v in phc.items() if v["count"]},
            "prism_speedup": round(value / conv_rate, 2),
            "prism_fp32_speedup": None,
            "map_rel_l2_vs_prism": float(np.linalg.norm(mc - gpu_map[idx]) / np.linalg.norm(gpu_map[idx])),
            "hbm": {"achieved": round(conv_bytes / dtc / 1e9, 1), "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                    "frac": round(conv_bytes / dtc / 1e9 / PEAK_HBM_GBPS, 4),
                    "byte_definition": ("read + write of 8 B x n_y x n_live_x per row or column pass of a "
                                        "wave, entrance waves, H once per chunk, new waves, exit band")},
        }

    return companion, inverse, conv


def crystal_finish(args, t_proc0, p, ps, ion, V, H, info, value, gpu_map, elapsed, ms_per_step, roofline,
                   roofline_fft, phases, companion, inverse, conv):
    """The FP32 leg (whole map unless --fp32-sample), the CPU sample and the JSON line."""
    import torch
    from paper_1908_07628_amd import eels
    out = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    # FP32 plain path
    if not args.fp32_sample:
        p32 = eels.Plan(p, precision="fp32")
        ws32 = p32.alloc_workspace()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p32.execute(V, H, out, ws32)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t1
        fp32 = {"value": p.n_probes / dt32, "ms_per_step": 1e3 * dt32, "measured_on": "the whole map",
                "split_rel_l2_vs_fp32": float(np.linalg.norm(gpu_map - out.cpu().numpy()) /
                                              np.linalg.norm(out.cpu().numpy()))}
        del ws32
    else:
        keep = np.isin(p.site_slice, ion[-args.fp32_slices:])
        p32 = eels.Plan(ps, precision="fp32")
        i32 = p32.info()
        ws32 = p32.alloc_workspace()
        p32.execute(V, H, out, ws32)        # warm the FP32 kernels
        torch.cuda.synchronize()
        eels.timing_enable(8192)
        p32.execute(V, H, out, ws32)
        torch.cuda.synchronize()
        ph32 = eels.timing_read()
        eels.timing_enable(0)
        contract_ms = sum(ph32[k]["ms"] for k in ("producer", "gemm1", "gemm2", "reduce", "gram"))
        scale = info["gemm_flops"] / i32["gemm_flops"]
        est_ms = phases["setup"] + phases["sweep"] + contract_ms * scale
        g1_32 = ph32["gemm1"]
        fp32 = {
            "value": p.n_probes / (est_ms * 1e-3), "ms_per_step": round(est_ms, 1),
            "measured_on": (f"contractions of the top {args.fp32_slices} of {len(ion)} ionised slices "
                            f"({int(keep.sum())} sites, {contract_ms:.0f} ms) scaled by GEMM work x{scale:.2f}; "
                            "set-up and sweeps from the full BF16-split step"),
            "gemm1_tflops": round(gemm1_flops(i32, ps) / (g1_32["ms"] * 1e-3) / 1e12, 1),
            "gemm1_frac_of_fp32_peak": round(gemm1_flops(i32, ps) / (g1_32["ms"] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4),
        }
        del ws32

    if conv is not None:
        conv["prism_fp32_speedup"] = round(fp32["value"] / conv["value"], 2)
    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "probe-px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16" if args.precision == "bf16_split" else args.precision,
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": [p.nx, p.ny], "n_slices": p.n_slices, "n_sites": p.n_sites,
                   "n_transitions": p.n_trans, "n_probes": p.n_probes, "N1": info["n_beams_in"],
                   "N2": info["n_beams_out"], "band_pixels": info["band_pixels"],
                   "precision": args.precision + " (hi+lo products, FP32 accumulate, FP64 map)"
                   if args.precision != "fp32" else "fp32", "contraction": "band basis, order S"},
        "roofline": roofline,
        "roofline_fft": roofline_fft,
        "companion_images": companion,
        "inverse_multislice": inverse,
        "conventional_multislice": conv,
        "phases_ms": phases,
        "fp32": fp32,
        "split_over_fp32": round(value / fp32["value"], 2),
    }
    if args.check:
        path = os.path.join(ROOT, "tests", "golden", "config2_samples.json")
        if os.path.exists(path):
            g = json.load(open(path))
            ref = np.array(g["map"])
            got = gpu_map[g["probe_index"]]
            result["check"] = {"max_abs_err_over_max": float(np.max(np.abs(got - ref)) / np.max(ref)),
                               "probes": g["probe_index"]}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        result["cpu_baseline"] = cpu_baseline(p)
    result["wall_s"] = round(time.time() - t_proc0, 1)
    return result


if __name__ == "__main__":
    main()
