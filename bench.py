"""EELS map throughput on one MI355X (probe positions per second).

Workload: the perovskite-crystal map (256 x 256 px over 20 x 20 A, 50 slices of 2 A,
650 ionised B sites x 9 transitions contracted over the full cell, 64 x 64 probes,
300 keV, 21 mrad aperture, 0-50 mrad detector).  A step is one complete map: set-up,
both scattering-matrix sweeps, every contraction and the FP64 reduction, with the
inputs already resident in HBM.

`value` is the BF16-split (hi+lo, FP32 accumulate) throughput.  The plain FP32 path
is reported beside it, measured on the contractions of a bounded subset of ionised
slices and scaled by GEMM work (see the `fp32` object); `--fp32-full` times it on the
whole map instead.  `roofline` is for the dominant kernel (the first contraction
GEMM), timed with HIP events on the execute stream.  `cpu_baseline` is the FP64
conventional-multislice oracle timed on a bounded sample of the same workload.

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


# sources whose change invalidates the committed counter figures (kernels and launch shapes)
TRAFFIC_SOURCES = ["kernels_gemm.hip", "kernels_sweep.hip", "fft_reg.h", "fft_lds.h", "plan.cpp"]


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
    }


def bench_serve(args):
    """Serving workload: Poisson arrivals, continuous batching, residency, p50/p99."""
    import torch
    import synth
    from paper_1908_07628_amd.serve import specimen_key
    t0 = time.time()
    pool = synth.specimen_pool(55, args.pool, (128, 256, 512, 1024), (10, 60), (1, 20), (16, 64), "req",
                               workers=min(16, os.cpu_count() or 1))
    log(f"{len(pool)} specimens generated in {time.time() - t0:.1f} s")
    keys = [specimen_key(p) for p in pool]
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
        serve_rates(args, pool, keys, free, prec, out)
        out["by_precision"][prec] = out["rates"]
    out["rates"] = out["by_precision"][precisions[0]]
    out["dtype"] = precisions[0]
    best = max(out["rates"].values(), key=lambda r: r["throughput_probe_px_s"])
    out["value"] = best["throughput_probe_px_s"]
    return out


def serve_rates(args, pool, keys, free, precision, out):
    """One Poisson stream per rate through a fresh server in the given precision."""
    import synth
    from paper_1908_07628_amd.serve import Server
    for rate in args.rates:
        reqs = synth.config5_stream(seed=5, rate_per_s=rate, n_requests=args.n_requests, pool=pool)
        srv = Server(int(0.8 * free), max_slots=4, precision=precision, residency=True)
        t0 = time.perf_counter()
        tickets = []
        for (t_arr, k, shift) in reqs:
            dt = t_arr - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            p = pool[k].replace(probes=pool[k].probes + shift)
            tickets.append(srv.submit(p, key=keys[k]))
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


NANO_WORKLOAD = ("nanoparticle 1024x1024 px over 100x100 A, 50 slices x 2 A: 80 A bcc sphere (22,659 atoms, "
                 "all ionised x 9 transitions) on a 20 A amorphous support (20,000 atoms); PRISM f = 4, 4 A crop "
                 "windows, 256x256 probes, 300 keV, 20 mrad aperture, 0-20 mrad detector")


def cpu_baseline_nanoparticle(p, info, sample_beams=3, sample_probes=1024):
    """FP64 PRISM oracle (one BLAS thread) on a bounded sample, scaled by its operation counts:
    `sample_beams` aperture beams swept to the deepest ionised slice and as many detector beams
    swept from the exit to the shallowest (the oracle sweeps every beam this way), and one
    site's contraction (oracle.prism.contract_windows) on windows of the real shapes with
    `sample_probes` eligible probes.  Full map = N_1 / sample_beams x S_1 sample + N_2 /
    sample_beams x S_2 sample + the contraction of every site, which is linear in its
    eligible-probe count."""
    import dataclasses
    import threadpoolctl
    from oracle import prism
    from oracle.common import make_setup, site_eligible
    ion = sorted(set(p.site_slice.tolist()))
    with threadpoolctl.threadpool_limits(1):
        t0 = time.perf_counter()
        st = make_setup(p.replace(probes=p.probes[:1], probe_shape=(1, 1)))
        t_setup = time.perf_counter() - t0
        b = slice(0, sample_beams)
        st1 = dataclasses.replace(st, ab1=st.ab1[b], ix1=st.ix1[b], iy1=st.iy1[b], C=st.C[b])
        t0 = time.perf_counter()
        prism.forward_s1(p, st1, [ion[-1]])
        t_s1 = time.perf_counter() - t0
        st2 = dataclasses.replace(st, ab2=st.ab2[b], ix2=st.ix2[b], iy2=st.iy2[b])
        t0 = time.perf_counter()
        for _ in prism.reverse_s2(p, st2, j_stop=ion[0]):
            pass
        t_s2 = time.perf_counter() - t0
        rng = np.random.default_rng(0)
        K, N1, N2 = info["k_pixels"], info["n_beams_in"], info["n_beams_out"]
        cplx = lambda *sh: rng.standard_normal(sh) + 1j * rng.standard_normal(sh)
        S1w, S2w, C = cplx(N1, K), cplx(N2, K), cplx(N1, sample_probes)
        Hs = [cplx(K) for _ in range(int(p.site_ntrans[0]))]
        t0 = time.perf_counter()
        prism.contract_windows(S1w, S2w, C, Hs, 16.0)
        t_site = time.perf_counter() - t0
    # mean eligible-probe count per site on the full raster (the oracle's f > 1 rule), over
    # a seeded sample of sites
    pick = np.random.default_rng(1).choice(p.n_sites, size=min(64, p.n_sites), replace=False)
    ps_mean = float(np.mean([np.sum(site_eligible(p, st, int(s))) for s in pick]))
    full = t_setup + (N1 * t_s1 + N2 * t_s2) / sample_beams + p.n_sites * t_site * ps_mean / sample_probes
    measured = t_setup + t_s1 + t_s2 + t_site
    return {
        "value": p.n_probes / full, "unit": "probe-px/s", "cores": 1, "kind": "oracle",
        "sample": (f"PRISM oracle FP64 (numpy FFT, one BLAS thread): set-up {t_setup:.1f} s, {sample_beams} "
                   f"aperture beams to slice {ion[-1]} {t_s1:.1f} s, {sample_beams} detector beams from the exit to "
                   f"slice {ion[0]} {t_s2:.1f} s, one site's contraction with {sample_probes} probes "
                   f"{t_site:.1f} s; scaled to "
                   f"{N1} + {N2} beams and {p.n_sites} sites x {ps_mean:.0f} eligible probes "
                   f"(estimated {full / 3600:.0f} h per map)"),
        "seconds_measured": round(measured, 1),
        "host_cpus": os.cpu_count(),
    }


def bench_nanoparticle(args):
    """Nanoparticle workload: the f = 4, 4 A-crop map (order P) at full size."""
    import torch
    import synth
    from paper_1908_07628_amd import eels
    t0 = time.time()
    p = synth.config3()
    log(f"inputs generated in {time.time() - t0:.1f} s: {p.n_sites} sites, {p.n_trans} transitions")
    V, H = eels.device_inputs(p)
    free, total = torch.cuda.mem_get_info()
    budget = int(free - (8 << 30))
    ion = sorted(set(p.site_slice.tolist()))

    # untimed warm-up on the top ionised slice (loads the kernels; not a step)
    small = subset_sites(p, np.nonzero(p.site_slice == ion[-1])[0])
    wplan = eels.Plan(small, precision=args.precision, max_workspace_bytes=budget)
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
        f"order={'S' if info['order'] == 1 else 'P'} groups={info['n_groups']} batches={info['n_batches']} "
        f"workspace={info['workspace_bytes'] / 1e9:.1f} GB (budget {budget / 1e9:.0f} GB)")
    for w in range(args.warmup):
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")
    eels.timing_enable(1 << 16)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    phase_tot = {}
    for k in range(args.steps):
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        for name, v in eels.timing_read().items():
            a = phase_tot.setdefault(name, {"ms": 0.0, "count": 0})
            a["ms"] += v["ms"]
            a["count"] += v["count"]
        log(f"step {k + 1}/{args.steps} done")
    elapsed = time.perf_counter() - t_start
    eels.timing_enable(0)
    value = p.n_probes * args.steps / elapsed
    gpu_map = out.cpu().numpy()
    del ws
    torch.cuda.empty_cache()
    phases = {k: round(v["ms"] / args.steps, 1) for k, v in phase_tot.items()}

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
    exec_factor = 3.0 if split else 1.0
    peak = PEAK_BF16_TFLOPS if split else PEAK_FP32_TFLOPS
    wgram = phase_tot.get("gram", {"count": 0})["count"] > 0
    kern = {"gemm1": ("first product Psi = C S_1w (k_cgemm_sc, store epilogue)", 8.0 * K * N1 * pairs,
                      "gemm1_traffic_bytes_per_site")}
    if wgram:
        kern["gemm2"] = ("G Psi product of the window-Gram form (k_cgemm_sc, complex64 store)", 8.0 * K * K * pairs,
                         "gpsi_traffic_bytes_per_site")
        kern["gram"] = ("Gram GEMM M = S_2w^H S_2w of the window-Gram form (k_cgemm_sc, Gram tiles)",
                        8.0 * N2 * K * (K + 1) / 2.0 * p.n_sites, "gram_traffic_bytes_per_site")
    else:
        kern["gemm2"] = ("second product (S_2w H_n) Psi (k_cgemm_sc, norm epilogue)" if split
                         else "second product (k_cgemm, norm epilogue)", 8.0 * N2 * K * nt * pairs,
                         "gemm2_traffic_bytes_per_site")
    cv = counter_values("k_cgemm_sc__nanoparticle_traffic_pmc.md") if split else {}
    contraction = {}
    for ph, (what, fl, _) in kern.items():
        t = phase_tot[ph]
        contraction[ph] = {"kernel": what, "ms": round(t["ms"] / args.steps, 1),
                           "useful_complex_tflops": round(fl * args.steps / (t["ms"] * 1e-3) / 1e12, 1),
                           "executed_frac": round(exec_factor * fl * args.steps / (t["ms"] * 1e-3) / 1e12 / peak, 4)}
    dom = max(kern, key=lambda k: phase_tot[k]["ms"])
    what, dom_flops, ckey = kern[dom]
    g = phase_tot[dom]
    n_launch = g["count"] / args.steps
    avg_ms = g["ms"] / max(g["count"], 1)
    per_launch = dom_flops / n_launch
    achieved = exec_factor * per_launch / (avg_ms * 1e-3) / 1e12
    # counter bytes per site of this kernel (profiling sample: the most populated slice, same
    # per-site shapes) times the full map's sites per launch
    traffic = cv[ckey] * p.n_sites / n_launch if ckey in cv else None
    roofline = {
        "bound": "mfma", "kernel": what,
        "achieved": round(achieved, 1), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
        "traffic": traffic, "avg_launch_ms": round(avg_ms, 3), "launches_per_step": n_launch,
        "algorithmic_flops_per_launch": exec_factor * per_launch,
        "useful_complex_tflops": round(per_launch / (avg_ms * 1e-3) / 1e12, 1),
        "flop_definition": ("3 BF16 MFMA products per complex multiply-add of the split algorithm, 8 real flops "
                            "each; useful = 8 M N K complex (Gram GEMM: its Hermitian half)" if split
                            else "8 M N K"),
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

    # FP32 on the top ionised slices (contractions scaled by GEMM work; set-up and sweeps
    # from the full step)
    ps = subset_sites(p, np.nonzero(np.isin(p.site_slice, ion[-args.fp32_slices:]))[0])
    p32 = eels.Plan(ps, precision="fp32", max_workspace_bytes=budget)
    i32 = p32.info()
    ws32 = p32.alloc_workspace()
    o32 = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    p32.execute(V, H, o32, ws32)
    torch.cuda.synchronize()
    eels.timing_enable(1 << 16)
    p32.execute(V, H, o32, ws32)
    torch.cuda.synchronize()
    ph32 = eels.timing_read()
    eels.timing_enable(0)
    del ws32
    contract_ms = sum(ph32[k]["ms"] for k in ("producer", "gemm1", "gemm2", "reduce", "gram"))
    scale = info["gemm_flops"] / i32["gemm_flops"]
    est_ms = phases["setup"] + phases["sweep"] + contract_ms * scale
    fp32 = {"value": p.n_probes / (est_ms * 1e-3), "ms_per_step": round(est_ms, 1),
            "measured_on": (f"contractions of the top {args.fp32_slices} ionised slices ({ps.n_sites} sites, "
                            f"{contract_ms:.0f} ms) scaled by GEMM work x{scale:.1f}; set-up and sweeps from "
                            "the full split step")}
    # the same sites in the split precision, against the FP32 map
    psp = eels.Plan(ps, precision=args.precision, max_workspace_bytes=budget)
    wsp = psp.alloc_workspace()
    osp = torch.empty(p.n_probes, dtype=torch.float64, device="cuda")
    psp.execute(V, H, osp, wsp)
    torch.cuda.synchronize()
    del wsp
    m32, msp = o32.cpu().numpy(), osp.cpu().numpy()
    fp32["split_rel_l2_vs_fp32"] = float(np.linalg.norm(msp - m32) / np.linalg.norm(m32))

    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "probe-px/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 1), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if args.precision == "bf16_split" else args.precision,
        "data": "synthetic",
        "config": {"workload": NANO_WORKLOAD, "grid": [p.nx, p.ny], "n_slices": p.n_slices, "n_sites": p.n_sites,
                   "n_transitions": p.n_trans, "n_probes": p.n_probes, "N1": N1, "N2": N2, "window_pixels": K,
                   "interp_f": p.interp_f, "slice_groups": info["n_groups"], "batches": info["n_batches"],
                   "workspace_GB": round(info["workspace_bytes"] / 1e9, 1),
                   "precision": args.precision + " (hi+lo products, FP32 accumulate, FP64 map)"
                   if split else "fp32",
                   "contraction": "cropped windows, order P" + (", window-Gram detector sum" if wgram else "")},
        "roofline": roofline, "contraction_kernels": contraction, "roofline_fft": roofline_fft,
        "phases_ms": phases, "fp32": fp32,
        "split_over_fp32": round(value / fp32["value"], 2),
        "map_sum": float(np.sum(gpu_map)),
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample ...")
        result["cpu_baseline"] = cpu_baseline_nanoparticle(p, info)
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--precision", default="bf16_split", choices=["bf16_split", "fp16_split", "fp32"])
    ap.add_argument("--fp32-full", action="store_true", help="time the FP32 path on the whole map")
    ap.add_argument("--fp32-slices", type=int, default=2, help="ionised slices of the FP32 sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true", help="compare sampled probes with the stored FP64 values")
    ap.add_argument("--workload", default="crystal", choices=["crystal", "nanoparticle", "batch", "serve"],
                    help="crystal: the benchmark map (default); nanoparticle: the f = 4 cropped-window map; "
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
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU layout is "
              "described in DESIGN.md and not run here.", file=sys.stderr)
        sys.exit(2)
    if args.profile_sample > 0:
        profile_sample(args)
        return
    if args.workload != "crystal":
        if args.precision == "bf16_split" and args.workload == "batch":
            args.precision = "fp16_split"
        res = {"batch": bench_batch, "serve": bench_serve, "nanoparticle": bench_nanoparticle}[args.workload](args)
        print(json.dumps(res), flush=True)
        return

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
    for w in range(args.warmup):
        plan.execute(V, H, out, ws)
        torch.cuda.synchronize()
        log(f"warmup step {w + 1}/{args.warmup} done")

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
    achieved = exec_factor * per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_BF16_TFLOPS if split else PEAK_FP32_TFLOPS
    roofline = {
        "bound": "mfma", "kernel": "k_cgemm_sc (first contraction GEMM)" if split else "k_cgemm",
        "achieved": round(achieved, 1), "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
        "traffic": counters.get("gemm1_traffic_bytes_per_launch") if split else None,
        "avg_launch_ms": round(avg_ms, 3),
        "launches_per_step": n_launch_per_step,
        "algorithmic_flops_per_launch": exec_factor * per_launch,
        "useful_complex_tflops": round(per_launch / (avg_ms * 1e-3) / 1e12, 1),
        "flop_definition": ("3 BF16 MFMA products per complex multiply-add of the split algorithm, "
                            "8 real flops each; useful = 8 M N K complex" if split else "8 M N K"),
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
    # Extras, on the sites of the top ionised slices (their costs do not grow with the site
    # count except the contractions): companion images (iBF with the EELS detector's angles,
    # ADF from 60 mrad to the band limit) computed with the map, and the inverse-multislice
    # S_1 (Sec. 4.C) against the exact path.
    ps = subset_sites(p, np.nonzero(np.isin(p.site_slice, ion[-args.fp32_slices:]))[0])
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

    # FP32 plain path
    if args.fp32_full:
        p32 = eels.Plan(p, precision="fp32")
        ws32 = p32.alloc_workspace()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p32.execute(V, H, out, ws32)
        torch.cuda.synchronize()
        dt32 = time.perf_counter() - t1
        fp32 = {"value": p.n_probes / dt32, "ms_per_step": 1e3 * dt32, "measured_on": "the whole map"}
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
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
