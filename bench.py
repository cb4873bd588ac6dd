"""Benchmark of the photon-migration hot path on one MI355X.

Workload: the 256^3 bicontinuous Cahn-wave mask at porosity 0.70 (|k| = 2 pi/24
per voxel, mask seed 0), solid mu_s = 0.5, mu_a = 0.01, g = 0.7 per voxel,
pores transparent, 1e8 photons per step, transport seed 20260809.  One step is
one full pass of the hot path: mc_run (zero tallies, pack the mask, persistent
walk) and mc_reduce (per-depth integer sums, FP64 estimators), with the mask
already resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "photon-steps/sec and photons/sec at 256^3 phi=0.70; batched vs plain"
HBM_PEAK_GBS = 8000.0
BYTES_PER_STEP = 8  # one int64 track-length deposit per photon-step
# the device sources the walk kernel is built from; counter summaries under profiles/ record their hash
SOURCES = ["include/photonmc.h", "paper_2604_13929_amd/csrc/batch.hip", "paper_2604_13929_amd/csrc/internal.hpp",
           "paper_2604_13929_amd/csrc/philox.hpp", "paper_2604_13929_amd/csrc/photonmc.hip",
           "paper_2604_13929_amd/csrc/walk.hpp"]
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "k_walk_plain_256cube_phi070_traffic.json")
FORMS_RECORD = os.path.join(ROOT, "profiles", "k_walk_batch_grad_counters.json")


def source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES:
        h.update(f.encode())
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(photons: int):
    """HBM bytes per walk launch from the committed counter summary, scaled to this
    launch's photon count, or None when the kernel sources changed since."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != source_sha256():
        return None
    return rec, rec["traffic_bytes_per_launch"] * photons / rec["photons"]


def plain_roofs(rec: dict, photons: int, photon_steps: int, walk_ms: float):
    """The plain walk's roofs for a launch of ``photons`` photons and ``photon_steps`` steps
    that took ``walk_ms``, from its committed counter record (same sources): the HBM-side
    bytes of the launch; the memory-side atomic request rate against the probe's ceiling
    for the walk's kind of request (the binding limit); and the VALU, at 4 cycles per
    wave64 instruction on each of the 1024 SIMDs at the clock the record's GRBM cycles and
    kernel time give (an estimate: FP64 and quarter-rate instructions take longer)."""
    scale = photons / rec["photons"]
    t = walk_ms * 1e-3
    traffic = rec["traffic_bytes_per_launch"] * scale
    req = rec["atomic_requests_per_launch"] * scale
    atomic = {"requests_per_launch": req, "requests_per_step": req / photon_steps,
              "achieved_requests_per_s": req / t,
              "ceiling_requests_per_s": rec["request_ceiling_per_s"], "ceiling": rec["request_ceiling_source"],
              "frac": req / t / rec["request_ceiling_per_s"],
              "source": os.path.relpath(TRAFFIC_RECORD, ROOT)}
    v = rec["valu"]
    clock = v["GRBM_GUI_ACTIVE"] / 8 / (rec["kernel_trace_avg_ms"] * 1e-3)   # one XCD's cycles per second
    simd_cycles = v["SQ_ACTIVE_INST_VALU"] * scale * 4 / 1024                 # VALU cycles per SIMD
    valu = {"instructions_per_step": v["SQ_INSTS_VALU"] / rec["photon_steps"],
            "thread_utilisation": v["thread_utilisation"],
            "roof_photon_steps_per_s": photon_steps / (simd_cycles / clock),
            "achieved_photon_steps_per_s": photon_steps / t,
            "frac": simd_cycles / (clock * t), "clock_hz": clock,
            "source": os.path.relpath(TRAFFIC_RECORD, ROOT)}
    return traffic, atomic, valu


def walk_roofline(form: str, photon_steps: int, walk_ms: float):
    """Roofline of the batched or differentiated walk launch just timed: the algorithmic
    HBM rate (8 B per photon-step) against 8 TB/s, and the memory-side atomic request
    rate (requests per launch from the committed counter record of the same workload)
    against the measured ceiling for those requests; None for the latter when the kernel
    sources changed since the counters were taken."""
    achieved = photon_steps * BYTES_PER_STEP / (walk_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "algorithmic_bytes_per_step": BYTES_PER_STEP, "atomic_request_roof": None}
    try:
        with open(FORMS_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return out
    if rec.get("source_sha256") != source_sha256():
        return out
    r = rec[form]
    req = r["atomic_requests_per_launch"] * photon_steps / r["photon_steps"]
    out["traffic"] = r["traffic_bytes_per_launch"] * photon_steps / r["photon_steps"]
    out["atomic_request_roof"] = {"requests_per_launch": req, "requests_per_step": req / photon_steps,
                                  "achieved_requests_per_s": req / (walk_ms * 1e-3),
                                  "ceiling_requests_per_s": rec["request_ceiling_per_s"],
                                  "frac": req / (walk_ms * 1e-3) / rec["request_ceiling_per_s"],
                                  "source": os.path.relpath(FORMS_RECORD, ROOT)}
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def batched_leg(args, seed):
    """The uneven 64-job batch: one persistent launch (autotuned, with the reductions)
    against the same 64 jobs as sequential plain runs (mc_run + mc_reduce each)."""
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    dev = torch.device("cuda:0")
    t0 = time.time()
    specs = inputs.batch_jobs(seed=0)
    jobs = []
    for j in specs:
        m = inputs.spinodal_mask_torch(j["nx"], j["ny"], j["nz"], j["wavelength"], j["porosity"],
                                       seed=j["mask_seed"], device=dev)
        jobs.append(pm.BatchJob(m, pm.Optics(j["mu_s"], j["mu_a"], j["g"]), j["n_photons"], seed,
                                stream_id=j["stream_id"]))
    torch.cuda.synchronize()
    n_total = sum(j.n_photons for j in jobs)
    vox = sum(j.mask.numel() for j in jobs)
    log(f"batch: 64 masks ({vox / 1e6:.0f} Mvoxels, {n_total / 1e6:.0f} M photons) built in {time.time() - t0:.1f}s")
    t0 = time.perf_counter()
    tuned = pm.autotune_batch(jobs)  # timed trials on a scaled-down copy; also stored in the tune cache
    t_tune = time.perf_counter() - t0
    log(f"batch autotune: {tuned} in {t_tune:.1f}s")
    b = pm.run_batch(jobs)           # warm-up, with the cached shape
    torch.cuda.synchronize()
    log("batch warm-up done")
    times, walk = [], []
    for i in range(args.batch_steps):
        del b
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b = pm.run_batch(jobs, timed=True)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
        walk.append(b.walk_ms)
        log(f"batch step {i}: {times[-1] * 1e3:.0f} ms (walk {b.walk_ms:.0f} ms)")
    steps = sum(int(r.scalars[pm.SCALARS.index("steps")].item()) for r in b.results)
    batch_scalars = [r.scalars.clone() for r in b.results]
    del b
    torch.cuda.synchronize()
    # the library's default launch shape on the same batch
    b = pm.run_batch(jobs, tune=pm.Tune(), timed=True)
    torch.cuda.synchronize()
    walk_default = b.walk_ms
    del b
    # the same batch keeping every job's escape-path histogram (Sec. 3.5 (c)) in the walk
    bins = [(4.0, 256)] * len(jobs)
    b = pm.run_batch(jobs, timed=True, escape_bins=bins)
    torch.cuda.synchronize()
    walk_esc = b.walk_ms
    esc_ok = all(int(r.escape_hist_n.sum()) == int(r.scalars[pm.SCALARS.index("esc_n")])
                 and int(r.escape_hist_w.sum()) == int(r.scalars[pm.SCALARS.index("esc_w")])
                 and torch.equal(r.scalars, c) for r, c in zip(b.results, batch_scalars))
    log(f"batch walk: default shape {walk_default:.0f} ms, with escape histograms {walk_esc:.0f} ms")
    del b
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    seq = []
    for j in jobs:
        r = pm.run(j.mask, j.optics, j.n_photons, j.seed, stream_id=j.stream_id)
        q, d, ws = pm.reduce_async(j.mask, r)
        seq.append(r.scalars)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t2
    log(f"sequential plain runs: {t_seq * 1e3:.0f} ms")
    identical = all(torch.equal(a, c) for a, c in zip(batch_scalars, seq))
    t_b = min(times)
    checks = None
    if not args.no_cpu:
        checks = batch_oracle_check(jobs, specs, seed)
    return {"oracle": checks,
            "workload": "64 Cahn-wave cubes, side U{64..256}, phi in {0.5..0.9}, mu_s [0.2,1], mu_a [0.005,0.05], "
                        "g [0.5,0.9], 1e6..1e7 photons each (seed 0)",
            "photons": n_total, "photon_steps": steps, "voxels": vox,
            "ms": t_b * 1e3, "walk_ms": min(walk), "photon_steps_per_s": steps / t_b, "photons_per_s": n_total / t_b,
            "sequential_plain_ms": t_seq * 1e3, "sequential_photon_steps_per_s": steps / t_seq,
            "speedup_vs_sequential": t_seq / t_b, "jobs_bitwise_equal_to_plain": identical,
            "autotuned_shape": {"block": tuned.block, "waves_per_cu": tuned.waves_per_cu, "chunk": tuned.chunk,
                                "refill": tuned.refill, "defer": tuned.defer, "tuning_s": t_tune},
            "walk_ms_default_shape": walk_default,
            "walk_ms_with_escape_histograms": walk_esc, "escape_histograms_consistent": esc_ok,
            "roofline": walk_roofline("batched", steps, min(walk))}


def batch_oracle_check(jobs, specs, seed, m=100_000):
    """Three jobs of the 64-job batch (the smallest cube, the largest, and the one with the
    highest mu_a) on their first m photon ids, through one batched launch, against the
    oracle on the same photons: relative errors of the estimators, R/T/A and steps."""
    import numpy as np
    import torch

    import oracle
    from oracle import estimators as est
    from paper_2604_13929_amd import photonmc as pm

    sizes = [s["nx"] * s["ny"] * s["nz"] for s in specs]
    pick = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), int(np.argmax([s["mu_a"] for s in specs]))})
    sub = [pm.BatchJob(jobs[k].mask, jobs[k].optics, m, seed, stream_id=jobs[k].stream_id) for k in pick]
    b = pm.run_batch(sub, tune=pm.Tune(256, 16, 256, 16))
    torch.cuda.synchronize()
    out = {}
    ncpu = len(os.sched_getaffinity(0))
    for i, k in enumerate(pick):
        mask_np = jobs[k].mask.cpu().numpy()
        o = jobs[k].optics
        t0 = time.perf_counter()
        ref = oracle.run(mask_np, o.mu_s, o.mu_a, o.g, m, seed, stream_id=jobs[k].stream_id, nthreads=ncpu)
        t_cpu = time.perf_counter() - t0
        tot = oracle.totals(ref)
        e = est.estimators(ref["fluence"][0], mask_np, m)
        s = b.summary(i)
        sc = b.results[i].scalar_dict()
        err = {q: abs(s[q] - e[q]) / abs(e[q]) for q in ("phi3d", "phi1d", "r") if np.isfinite(e[q]) and e[q] != 0}
        err.update({q: abs(sc[q] - tot[q]) / (m * pm.W1) for q in ("R", "T", "A")})
        err["steps"] = abs(sc["steps"] - tot["steps"]) / tot["steps"]
        out[f"job{k}"] = {"side": specs[k]["nx"], "porosity": specs[k]["porosity"],
                          "optics": [specs[k]["mu_s"], specs[k]["mu_a"], specs[k]["g"]], "photons": m,
                          "relative_error": err, "oracle_s": t_cpu}
        log(f"batch job {k} vs oracle ({m} photons): " + ", ".join(f"{q} {v:.1e}" for q, v in err.items()))
    return out


def morphology_leg(args, seed):
    """512 x 512 x 256 mask at phi = 0.90 next to the homogeneous slab of the same
    thickness with (1 - phi)-scaled coefficients: RMS_w of the depth profiles and the
    in-void path statistics of escaping photons."""
    import numpy as np
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    wl = inputs.WORKLOADS["M3"]
    n = args.photons
    d3 = inputs.spinodal_mask_torch(wl["nx"], wl["ny"], wl["nz"], wl["wavelength"], wl["porosity"], seed=0)
    dh = torch.zeros_like(d3)
    base = pm.Optics(**inputs.SOLID_OPTICS)
    phi = wl["porosity"]
    opt_h = pm.Optics(float(np.float32((1 - phi) * base.mu_s)), float(np.float32((1 - phi) * base.mu_a)), base.g)
    out = {}
    for name, d, opt in (("M3", d3, base), ("H3", dh, opt_h)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pm.run(d, opt, n, seed, timed=True)
        s = pm.reduce(d, r)
        t = time.perf_counter() - t0
        out[name] = {"ms": t * 1e3, "walk_ms": r.walk_ms, "photon_steps_per_s": s["steps_per_photon"] * n / t,
                     "photons_per_s": n / t, "depth": s.depth, "summary": s}
        log(f"{name}: {t * 1e3:.0f} ms, {s['steps_per_photon']:.0f} steps/photon")
    sm, sh = out["M3"]["summary"], out["H3"]["summary"]
    # Eq. RMSw with Table S1's variants: the spinodal slab and the homogeneous slab each
    # against the collimated diffusion approximation of their common effective medium
    # (Sec. 2.4), and the spinodal slab against the homogeneous one
    da, da_lopt = pm.da_profile(base.mu_s, base.mu_a, base.g, phi, wl["nz"])
    rms = {"M3_vs_H3": pm.rms_w(out["M3"]["depth"], out["H3"]["depth"]),
           "M3_vs_DA": pm.rms_w(out["M3"]["depth"], da), "H3_vs_DA": pm.rms_w(out["H3"]["depth"], da)}
    log("RMS: " + "; ".join(f"{k} {v['weighted']:.4f} (unweighted {v['unweighted']:.4f}, log {v['log']:.4f})"
                            for k, v in rms.items()))
    checks = {}
    if not args.no_cpu:
        ncpu = len(os.sched_getaffinity(0))
        checks = {"M3": oracle_check(d3.cpu().numpy(), d3, base, 1_000_000, seed, ncpu),
                  "H3": oracle_check(dh.cpu().numpy(), dh, opt_h, 1_000_000, seed, ncpu)}
    return {"oracle": checks,
            "workload": "512x512x256 Cahn-wave mask phi=0.90 (lambda 32) vs homogeneous slab mu_s 0.05 mu_a 0.001 g 0.7, "
                        f"{n:.0e} photons each",
            "rms_w_M3_vs_H3": rms["M3_vs_H3"]["weighted"], "rms": rms,
            "L_opt": {"M3": sm["L_opt"], "H3": sh["L_opt"], "DA": da_lopt},
            "front_back": {"M3": sm["front_back"], "H3": sh["front_back"], "DA": float(da[0] / da[-1])},
            "Pw_void_gt_L": sm["Pw_void_gtL"], "Pn_void_gt_L": sm["Pn_void_gtL"],
            "mean_void_path_escaping": sm["mean_void_path"], "escaping_weight_fraction": sm["esc_frac"],
            "phi3d": {"M3": sm["phi3d"], "H3": sh["phi3d"]}, "phi1d": {"M3": sm["phi1d"], "H3": sh["phi1d"]},
            "r_M3": sm["r"], "R_T_A_M3": [sm["R"], sm["T"], sm["A"]], "R_T_A_H3": [sh["R"], sh["T"], sh["A"]],
            "photon_steps_per_s": {k: out[k]["photon_steps_per_s"] for k in out},
            "ms": {k: out[k]["ms"] for k in out}}


def oracle_kw(opt) -> dict:
    """The oracle's boundary-model arguments for the binding's optics."""
    return dict(boundary=opt.boundary, lateral=opt.lateral, n_solid=opt.n_solid if opt.n_solid else 1.0,
                gate=opt.gate if opt.gate > 0 else float("inf"))


def oracle_check(mask_np, dmask, opt, m, seed, ncpu):
    """The oracle on the first ``m`` photon ids of a workload and the GPU on the same
    ids: relative errors of the estimators, and the oracle's time."""
    import math

    import oracle
    from oracle import estimators as est
    from paper_2604_13929_amd import photonmc as pm

    t0 = time.perf_counter()
    ref = oracle.run(mask_np, opt.mu_s, opt.mu_a, opt.g, m, seed, nthreads=ncpu, **oracle_kw(opt))
    t_cpu = time.perf_counter() - t0
    tot = oracle.totals(ref)
    sub = pm.run(dmask, opt, m, seed)
    ssum = pm.reduce(dmask, sub)
    e = est.estimators(ref["fluence"][0], mask_np, m)
    err = {k: abs(ssum[k] - e[k]) / abs(e[k]) for k in ("phi3d", "phi1d", "r")
           if math.isfinite(e[k]) and e[k] != 0}
    gsc = sub.scalar_dict()
    for k in ("R", "T", "A", "gated"):
        err[k] = abs(gsc[k] - tot[k]) / (m * pm.W1)
    err["steps"] = abs(gsc["steps"] - tot["steps"]) / tot["steps"]
    return {"photons": m, "relative_error": err, "oracle_s": t_cpu,
            "oracle_photon_steps_per_s": tot["steps"] / t_cpu}


def rows_leg(args, seed, field):
    """The two other single-mask workloads, each timed on the GPU and
    (unless --no-cpu) checked against the oracle on its first photon ids: 32^3
    phi = 0.70 (all 1e5 photons) and 256^3 phi = 0.90 thresholded from the plain
    workload's field (1e8 photons)."""
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    ncpu = len(os.sched_getaffinity(0))
    opt = pm.Optics(**inputs.SOLID_OPTICS)
    w1 = inputs.WORKLOADS["M1"]
    m1 = inputs.spinodal_mask(w1["nx"], w1["ny"], w1["nz"], w1["wavelength"], w1["porosity"],
                              seed=inputs.PAPER_MASK_SEED)
    m2b = inputs.rank_threshold(field, inputs.WORKLOADS["M2b"]["porosity"])
    rows = {}
    for name, mask_np, n, m_cpu in (("M1_32cube_phi070", m1, w1["n_photons"], w1["n_photons"]),
                                    ("M2b_256cube_phi090", m2b, args.photons, 1_000_000)):
        d = torch.from_numpy(mask_np).cuda()
        pm.run(d, opt, min(n, 1 << 20), seed)          # warm the code path and the allocator
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pm.run(d, opt, n, seed, timed=True)
        s = pm.reduce(d, r)
        t = time.perf_counter() - t0
        steps = s["steps_per_photon"] * n
        row = {"photons": n, "ms": t * 1e3, "walk_ms": r.walk_ms, "photon_steps_per_s": steps / t,
               "photons_per_s": n / t, "phi3d": s["phi3d"], "phi1d": s["phi1d"], "r": s["r"],
               "R_T_A": [s["R"], s["T"], s["A"]], "steps_per_photon": s["steps_per_photon"]}
        if not args.no_cpu:
            row["oracle"] = oracle_check(mask_np, d, opt, m_cpu, seed, ncpu)
        log(f"{name}: {t * 1e3:.1f} ms, {steps / t:.3e} steps/s")
        rows[name] = row
    return rows


def paper_leg(args, seed, mask_np, mask):
    """The paper's own boundary model (one-voxel air pads, lateral mirrors, solid index
    n_eff = 1.746 with Fresnel reflection and refraction, gate of Eq. tend) on the plain
    workload's 256^3 phi = 0.70 mask: with the paper's shell optics per 1.45 um voxel
    (mu_s = 20118 1/m, mu_a = 5159 1/m, g = 0), and with the plain workload's optics."""
    import numpy as np
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    def f32(x):
        return float(np.float32(x))

    a_vox, nz, phi = 1.45e-6, mask_np.shape[0], float(mask_np.mean())
    n = args.photons
    shell = dict(mu_s=f32(20118.0 * a_vox), mu_a=f32(5159.0 * a_vox), g=0.0)
    plain = dict(inputs.SOLID_OPTICS)
    out = {}
    for name, o in (("paper_optics", shell), ("plain_optics", plain)):
        gate = pm.time_gate_voxels(o["mu_s"], o["mu_a"], o["g"], phi, nz, 1.746)
        opt = pm.paper_optics(o["mu_s"], o["mu_a"], o["g"], n_solid=f32(1.746), lateral=pm.LATERAL_MIRROR,
                              gate=gate)
        pm.run(mask, opt, 1 << 20, seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = pm.run(mask, opt, n, seed, timed=True)
        s = pm.reduce(mask, r)
        t = time.perf_counter() - t0
        steps = s["steps_per_photon"] * n
        row = {"optics": {**o, "n_solid": 1.746, "lateral": "mirror", "gate_voxels": gate, "air_pads": 1},
               "photons": n, "ms": t * 1e3, "walk_ms": r.walk_ms, "photon_steps_per_s": steps / t,
               "photons_per_s": n / t, "R": s["R"], "T": s["T"], "A": s["A"], "gated": s["gated"],
               "phi3d": s["phi3d"], "phi1d": s["phi1d"], "r": s["r"], "ratio": s["ratio"],
               "steps_per_photon": s["steps_per_photon"], "closure_exact": s["closure_exact"]}
        if not args.no_cpu:
            row["oracle"] = oracle_check(mask_np, mask, opt, 100_000, seed, len(os.sched_getaffinity(0)))
        log(f"paper model, {name}: {t * 1e3:.0f} ms, {steps / t:.3e} steps/s, r {s['r']:.4f}")
        out[name] = row
    return {"workload": "256^3 Cahn-wave mask phi=0.70 (lambda 24), air pads, lateral mirrors, n_solid 1.746 "
                        "(Fresnel), gate of Eq. tend, 1e8 photons", **out}


def ch_leg(args):
    """The Cahn-Hilliard generator (Eq. CH_spectral, App. A) on the paper's domain,
    384 x 1024 x 1024 voxels, kappa_CH = 0.1140, dt = 0.0450, from the App. A initial
    field (0.5 + N(0, 0.05^2), clipped, seed 0): one stopping-check interval of
    `ch_steps` steps timed with HIP events, plus the PSD check; the numpy oracle's
    rate on a 64^3 grid as the CPU reference."""
    import numpy as np
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import spinodal as sp

    nz, ny, nx = 384, 1024, 1024
    g = sp.grid_from_target(nx, ny, nz, 17.4 / 1.45)
    kappa, dt = g.kappa, g.dt
    dev = torch.device("cuda:0")
    t0 = time.time()
    phi0 = torch.from_numpy(inputs.ch_initial_field(nx, ny, nz, seed=inputs.PAPER_MASK_SEED)).to(dev)
    log(f"CH initial field {nz}x{ny}x{nx} built in {time.time() - t0:.1f}s")
    ws = sp.workspace(g, dev)
    st = sp.init(phi0, g, ws)
    del phi0
    sp.steps(st, g, 4, ws)
    torch.cuda.synchronize()
    n = args.ch_steps
    t1 = time.perf_counter()
    ms = sp.steps(st, g, n, ws, timed=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    t2 = time.perf_counter()
    p = sp.psd(st, g, ws)
    size = sp.dominant_size(p, g)
    torch.cuda.synchronize()
    psd_ms = (time.perf_counter() - t2) * 1e3
    spec_bytes = nz * ny * (nx // 2 + 1) * 16
    bytes_per_step = 10 * spec_bytes
    voxels = nx * ny * nz
    log(f"CH: {n} steps in {ms:.0f} ms ({ms / n:.2f} ms/step, {bytes_per_step / (ms / n * 1e-3) / 1e9:.0f} GB/s)")
    out = {"workload": "Cahn-Hilliard semi-implicit spectral steps, 384x1024x1024 FP64, kappa 0.1140, dt 0.0450",
           "steps": n, "ms": ms, "wall_ms": wall * 1e3, "ms_per_step": ms / n, "steps_per_s": n / (ms * 1e-3),
           "voxel_steps_per_s": voxels * n / (ms * 1e-3),
           "roofline": {"bound": "hbm", "bytes_per_step": bytes_per_step,
                        "achieved": bytes_per_step / (ms / n * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": bytes_per_step / (ms / n * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "note": "ten spectrum-sized (complex FP64 [nz][ny][nx/2+1]) transfers per step"},
           "psd_ms": psd_ms, "dominant_size_voxels_after": size, "steps_done": n + 4}
    if not args.no_cpu:
        from oracle import cahn_hilliard as och
        kappa = och.kappa_from_target(17.4 / 1.45)
        dt = och.dt_from_kappa(kappa)
        m = 64
        phi_s = inputs.ch_initial_field(m, m, m, seed=1)
        ph = och.spectrum(phi_s)
        och.steps(ph, phi_s.shape, 2, dt, kappa)
        t3 = time.perf_counter()
        k = 50
        och.steps(ph, phi_s.shape, k, dt, kappa)
        tc = time.perf_counter() - t3
        out["cpu_baseline"] = {"value": m ** 3 * k / tc, "unit": "voxel-steps/s", "kind": "oracle",
                               "sample": f"{k} steps on a {m}^3 grid, numpy FFT (single thread)", "seconds": tc}
        out["gpu_over_cpu"] = out["voxel_steps_per_s"] / out["cpu_baseline"]["value"]
    del st, ws
    torch.cuda.empty_cache()
    return out


def analytics_leg(args, seed, mask_np, mask):
    """The Sec. 3.5 analytics on the tally of one paper-model run (configuration P with
    the paper's shell optics, 1e8 photons) over the 256^3 phi = 0.70 mask: chord
    histograms on all three axes, the pore distance transform, the brightest-decile
    co-localisation and the pore-phase Spearman correlation on deep slices
    (z >= 0.1 mm = slice 69 at 1.45 um voxels), the mask's radial PSD, the
    depth-normalised phase contrast, and escape-path histograms: kept by the run's own walk
    over all its photons, and from 1e7 traced photons.  Each call timed with events on
    torch's current stream (the one the bindings launch on), warm (second call); the
    oracle's co-localisation and Spearman on the same tally as the CPU reference and
    parity check."""
    import numpy as np
    import torch

    from paper_2604_13929_amd import analytics as an
    from paper_2604_13929_amd import photonmc as pm
    from paper_2604_13929_amd import spinodal as sp

    def f32(x):
        return float(np.float32(x))

    a_vox, nz, phi = 1.45e-6, mask_np.shape[0], float(mask_np.mean())
    o = dict(mu_s=f32(20118.0 * a_vox), mu_a=f32(5159.0 * a_vox), g=0.0)
    gate = pm.time_gate_voxels(o["mu_s"], o["mu_a"], o["g"], phi, nz, 1.746)
    opt = pm.paper_optics(o["mu_s"], o["mu_a"], o["g"], n_solid=f32(1.746), lateral=pm.LATERAL_MIRROR, gate=gate)
    n = args.photons
    esc_width, esc_bins = 4.0, 256
    res = pm.run(mask, opt, n, seed, escape_bins=(esc_width, esc_bins), timed=True)
    _, depth, _ = pm.reduce_async(mask, res)
    F = res.fluence
    torch.cuda.synchronize()
    z0 = int(math.ceil(0.1e-3 / a_vox))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        out = fn()
        e1.record()
        e1.synchronize()
        return out, e0.elapsed_time(e1)

    out = {"workload": "analytics of Sec. 3.5 on the paper-model tally (256^3 phi=0.70, paper optics, 1e8 photons)",
           "deep_slice_z0": z0, "ms": {}}
    hists = {}
    for axis, name in ((0, "x"), (1, "y"), (2, "z")):
        hists[name], out["ms"][f"chords_{name}"] = timed(lambda: an.chord_histogram(mask, axis))
    hz = hists["z"].cpu().numpy().astype(np.float64)
    lengths = np.arange(hz.shape[1], dtype=np.float64)
    half = nz // 2
    out["chords_z"] = {"mean_pore": float((lengths * hz[1]).sum() / hz[1].sum()),
                       "mean_solid": float((lengths * hz[0]).sum() / hz[0].sum()),
                       f"plen_pore_gt_{half}": float((lengths * hz[1])[lengths > half].sum() / (lengths * hz[1]).sum())}
    dist, out["ms"]["pore_distance"] = timed(lambda: an.pore_distance(mask))
    voxels = mask_np.size
    # algorithmic bytes of the transform: mask read, g written, two envelope passes read and write g,
    # the output pass reads g and writes the FP64 distance: 1 + 4 + 2 * 8 + 12 bytes per voxel
    edt_bytes = 33 * voxels
    out["pore_distance_gbs"] = edt_bytes / (out["ms"]["pore_distance"] * 1e-3) / 1e9
    dn = dist.cpu().numpy()
    out["mean_pore_distance_voxels"] = float(dn[mask_np == 1].mean())
    del dist
    (kk, ks), out["ms"]["bright_colocalization"] = timed(lambda: an.bright_colocalization(mask, F, z0, 0.1))
    frac_solid = ks.cpu().numpy() / kk.cpu().numpy()
    out["bright_decile_solid_fraction"] = {"mean": float(frac_solid.mean()), "sd": float(frac_solid.std(ddof=1)),
                                           "solid_volume_fraction": 1.0 - phi, "slices": int(frac_solid.size)}
    (rho, npore), out["ms"]["pore_spearman"] = timed(lambda: an.pore_spearman(mask, F, z0))
    r = rho.cpu().numpy()
    out["pore_spearman"] = {"mean": float(np.nanmean(r)), "sd": float(np.nanstd(r, ddof=1)),
                            "slices": int(np.isfinite(r).sum())}
    psd, out["ms"]["mask_psd"] = timed(lambda: an.mask_psd(mask))
    s_peak, size = sp.psd_peak(psd, max(mask_np.shape))
    out["mask_psd"] = {"peak_shell": s_peak, "dominant_size_voxels": size}
    pc, out["ms"]["phase_contrast"] = timed(lambda: an.phase_contrast(depth, 0))
    out["phase_contrast"] = {k: float(v) for k, v in pc.items()}
    m_tr = 10_000_000
    thr = (float(nz), 0.5 * nz)
    eh, out["ms"]["escape_paths_trace_and_bin"] = timed(
        lambda: an.escape_paths(mask, opt, m_tr, seed, bin_width=4.0, nbins=256, thresholds=thr))
    aw = eh["above_w"].cpu().numpy()
    esc_w = int(eh["hist_w"].sum().item())
    out["escape_paths"] = {"photons": m_tr, "escaped_weight_fraction": esc_w / (m_tr * pm.W1),
                           "weight_fraction_void_path_gt_L": float(aw[0]) / esc_w if esc_w else None,
                           "weight_fraction_void_path_gt_L2": float(aw[1]) / esc_w if esc_w else None}
    del eh
    # the same histogram over all n photons, kept by the walk that made the tally
    hw = res.escape_hist_w.cpu().numpy().astype(np.float64)
    esc_all = hw.sum()
    lo_l, lo_l2 = int(nz / esc_width), int(0.5 * nz / esc_width)
    out["escape_paths_run"] = {"photons": n, "walk_ms_with_histogram": res.walk_ms, "bin_width": esc_width,
                               "nbins": esc_bins, "escaped_weight_fraction": esc_all / (n * pm.W1),
                               "weight_fraction_void_path_ge_L": float(hw[lo_l:].sum() / esc_all) if esc_all else None,
                               "weight_fraction_void_path_ge_L2": float(hw[lo_l2:].sum() / esc_all) if esc_all else None}
    log("analytics: " + ", ".join(f"{k} {v:.2f} ms" for k, v in out["ms"].items()))
    log(f"analytics: walk with the escape histogram {res.walk_ms:.1f} ms for {n} photons")
    if not args.no_cpu:
        from oracle import analytics as oan
        Fn = F.cpu().numpy()
        t0 = time.perf_counter()
        kw, sw = oan.bright_colocalization(Fn, mask_np, z0, 0.1)
        t1 = time.perf_counter()
        rw, nw = oan.pore_spearman(Fn, mask_np, z0)
        t2 = time.perf_counter()
        ok = np.isfinite(rw)
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "unit": "ms",
                               "bright_colocalization_ms": (t1 - t0) * 1e3,
                               "pore_spearman_ms": (t2 - t1) * 1e3,
                               "sample": "the same tally and mask; numpy stable argsort per slice, scipy EDT and "
                                         "spearmanr per slice"}
        out["oracle_match"] = {"bright_colocalization_exact": bool(np.array_equal(ks.cpu().numpy(), sw)
                                                                   and np.array_equal(kk.cpu().numpy(), kw)),
                               "pore_spearman_max_abs_diff": float(np.abs(r[ok] - rw[ok]).max()),
                               "pore_spearman_nan_pattern_equal": bool(np.array_equal(np.isfinite(r), ok)),
                               "pore_counts_exact": bool(np.array_equal(npore.cpu().numpy(), nw))}
        log(f"analytics oracle: decile {(t1 - t0) * 1e3:.0f} ms, spearman {(t2 - t1) * 1e3:.0f} ms, "
            f"match {out['oracle_match']}")
    del F, res
    torch.cuda.empty_cache()
    return out


def grad_oracle_check(seed, n=100_000, B=32):
    """GPU likelihood-ratio Jacobian (FP32 transport) on the 32^3 workload against the
    oracle's FP64 likelihood-ratio bins on the same photons: z-scores with the
    oracle's spread over B photon batches."""
    import numpy as np
    import torch

    import oracle
    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    w1 = inputs.WORKLOADS["M1"]
    m1 = inputs.spinodal_mask(w1["nx"], w1["ny"], w1["nz"], w1["wavelength"], w1["porosity"],
                              seed=inputs.PAPER_MASK_SEED)
    opt = pm.Optics(**inputs.SOLID_OPTICS)
    g = pm.grad(torch.from_numpy(m1).cuda(), opt, n, seed)
    jac = g.jac.cpu().numpy()[:, :2]
    ref = oracle.run(m1, opt.mu_s, opt.mu_a, opt.g, n, seed, nbatch=B, grad=True, fluence=False,
                     nthreads=len(os.sched_getaffinity(0)))
    nz, ny, nx = m1.shape
    per_b = ref["grad"] * (nx * ny) / (n / B * pm.W1)            # [B, 3, 2, nz]
    d3 = per_b[:, :, 0, :].sum(-1) / (m1 == 0).sum()
    d1 = per_b.sum(axis=(2, 3)) / m1.size
    want = np.stack([d3.mean(0), d1.mean(0)], 1)                 # [3, 2]
    sig = np.stack([d3.std(0, ddof=1), d1.std(0, ddof=1)], 1) / np.sqrt(B)
    return {"photons": n, "gpu": jac.tolist(), "oracle": want.tolist(),
            "z": ((jac - want) / sig).tolist(), "rows": ["mu_s", "mu_a", "g"], "columns": ["d_phi3d", "d_phi1d"]}


def grad_leg(args, seed, mask):
    """Likelihood-ratio Jacobian on the plain workload and its check against
    central finite differences with common random numbers (relative step 1e-3),
    with the spread of 8 photon sub-ranges as the error."""
    import numpy as np
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    n = args.photons
    base = pm.Optics(**inputs.SOLID_OPTICS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = pm.grad(mask, base, n, seed, timed=True)
    jac = g.jac.cpu().numpy()
    t_lr = time.perf_counter() - t0
    steps = int(g.run.scalars[pm.SCALARS.index("steps")].item())
    log(f"grad: {t_lr * 1e3:.0f} ms (walk {g.walk_ms:.0f} ms)")
    B, h = 8, 1e-3
    chunk = n // B
    lr = np.stack([pm.grad(mask, base, chunk, seed, photon_begin=b * chunk).jac.cpu().numpy()[:, :2]
                   for b in range(B)])
    res = {}
    names = ("mu_s", "mu_a", "g")
    for pi, name in enumerate(names):
        vals = {"mu_s": base.mu_s, "mu_a": base.mu_a, "g": base.g}
        plus, minus = dict(vals), dict(vals)
        plus[name] = float(np.float32(vals[name] * (1 + h)))
        minus[name] = float(np.float32(vals[name] * (1 - h)))
        fd = []
        for b in range(B):
            rp = pm.reduce(mask, pm.run(mask, pm.Optics(**plus), chunk, seed, photon_begin=b * chunk))
            rm = pm.reduce(mask, pm.run(mask, pm.Optics(**minus), chunk, seed, photon_begin=b * chunk))
            fd.append([(rp[k] - rm[k]) / (plus[name] - minus[name]) for k in ("phi3d", "phi1d")])
        fd = np.array(fd)
        fm, fs = fd.mean(0), fd.std(0, ddof=1) / np.sqrt(B)
        lm, ls = lr[:, pi].mean(0), lr[:, pi].std(0, ddof=1) / np.sqrt(B)
        res[name] = {"lr": jac[pi, :2].tolist(), "lr_subrange_mean": lm.tolist(), "lr_sigma": ls.tolist(),
                     "fd": fm.tolist(), "fd_sigma": fs.tolist(), "z": ((fm - lm) / np.hypot(fs, ls)).tolist()}
        log(f"grad check {name}: LR {lm} FD {fm} z {res[name]['z']}")
    check = None
    if not args.no_cpu:
        check = grad_oracle_check(seed)
    return {"oracle_lr_32cube": check,
            "workload": "plain workload, d<Phi>_3D and d<Phi>_1D (and dPhi(z)) wrt solid mu_s, mu_a, g",
            "ms": t_lr * 1e3, "walk_ms": g.walk_ms, "photon_steps_per_s": steps / t_lr, "photons_per_s": n / t_lr,
            "check_vs_crn_fd": res, "fd_relative_step": h, "subranges": B,
            "columns": ["d_phi3d", "d_phi1d"], "roofline": walk_roofline("differentiated", steps, g.walk_ms)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=100_000_000)
    ap.add_argument("--cpu-photons", type=int, default=3_000_000, help="oracle sample size (first ids)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-morph", action="store_true")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="skip the 32^3 and phi = 0.90 rows")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper boundary model rows")
    ap.add_argument("--no-ch", action="store_true", help="skip the Cahn-Hilliard generator leg")
    ap.add_argument("--no-analytics", action="store_true", help="skip the Sec. 3.5 analytics leg")
    ap.add_argument("--ch-steps", type=int, default=200)
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--defer", type=int, default=0, help="interaction deferral of the plain walk (0: library default)")
    ap.add_argument("--waves-per-cu", type=int, default=0, help="resident waves per CU of the plain walk (0: default)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--scatter-probe", action="store_true",
                    help="only measure random 64-bit scatter / atomic throughput (the deposit roofline)")
    ap.add_argument("--hot-probe", action="store_true",
                    help="only measure atomic throughput onto few addresses (64 to 262144 table entries)")
    args = ap.parse_args()
    if args.scatter_probe:
        import torch

        from paper_2604_13929_amd import photonmc as pm
        pm.load()
        out = {}
        names = {0: "atomic64_device", 1: "atomic64_workgroup", 2: "store64", 3: "atomic32_device",
                 4: "atomic64_device_wave_contiguous", 5: "atomic64_device_16lane_128B",
                 6: "atomic64_device_8lane_64B", 7: "atomic64_device_4lane_32B", 8: "atomic64_device_return",
                 9: "atomic32_device_return", 10: "atomic32_device_16lane_64B",
                 11: "atomic32_device_16lane_64B_return", 12: "atomic64_device_8lane_64B_return"}
        # every mode at 16 waves per CU on four table sizes, the walk's request kinds also at 64, 192
        # and 256 MiB (the staging tallies of the 256^3 workload in lines and in planes, and of the
        # 512x512x256 volumes), then the occupancy sweep at 128 MiB
        plan = [(mib, mode, 16) for mib in (2, 128, 512, 2048) for mode in names]
        plan += [(mib, mode, 16) for mib in (64, 192, 256) for mode in (0, 3, 6, 10, 11)]
        plan += [(128, mode, w) for w in (4, 8, 24, 32) for mode in (0, 3, 6, 8, 9, 10, 11, 12)]
        tables = {}
        for mib, mode, w in plan:
            if mib not in tables:
                tables.clear()
                torch.cuda.empty_cache()
                tables[mib] = torch.zeros(mib * 1024 * 1024 // 8, dtype=torch.int64, device="cuda:0")
            t = tables[mib]
            pm.probe_scatter(t, 1 << 24, mode, w)
            key = f"{names[mode]}_{mib}MiB_{w}w"
            out[key] = pm.probe_scatter(t, 1 << 30, mode, w)
            log(f"{mib:5d} MiB {w:2d} waves/CU {names[mode]:36s} {out[key] / 1e9:8.2f} G ops/s")
        print(json.dumps({"scatter_probe_ops_per_s": out}))
        return
    if args.hot_probe:
        import torch

        from paper_2604_13929_amd import photonmc as pm
        pm.load()
        out = {}
        names = {0: "atomic64_device", 8: "atomic64_device_return", 3: "atomic32_device"}
        for entries in (64, 512, 4096, 32768, 262144):
            t = torch.zeros(entries, dtype=torch.int64, device="cuda:0")
            for mode in names:
                pm.probe_scatter(t, 1 << 20, mode, 16)
                key = f"{names[mode]}_{entries}entries"
                out[key] = pm.probe_scatter(t, 1 << 26, mode, 16)
                log(f"{entries:7d} entries ({entries * 8 // 64:5d} lines) {names[mode]:24s} "
                    f"{out[key] / 1e9:8.3f} G ops/s")
        print(json.dumps({"hot_probe_ops_per_s": out}))
        return
    if args.copy_probe:
        import torch
        x = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")   # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": x.numel() * 8}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU sharding is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_13929_amd import inputs
    from paper_2604_13929_amd import photonmc as pm

    assert torch.cuda.is_available(), "bench needs a GPU"
    pm.load()
    dev = torch.device("cuda:0")
    wl = inputs.WORKLOADS["M2a"]
    t0 = time.time()
    field = inputs.cahn_field(wl["nx"], wl["ny"], wl["nz"], wl["wavelength"], inputs.PAPER_MASK_SEED)
    mask_np = inputs.rank_threshold(field, wl["porosity"])
    log(f"mask {mask_np.shape} porosity {mask_np.mean():.6f} built in {time.time() - t0:.1f}s")
    # the mask's host-to-device copy, outside the timed steps (reported on its own): pinned
    # staging, then one copy timed with events on the current stream
    pinned = torch.from_numpy(mask_np).pin_memory()
    mask = torch.empty(mask_np.shape, dtype=torch.uint8, device=dev)
    mask.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    mask.copy_(pinned, non_blocking=True)
    e1.record()
    e1.synchronize()
    h2d_ms = e0.elapsed_time(e1)
    del pinned
    opt = pm.Optics(**inputs.SOLID_OPTICS)
    seed = inputs.PAPER_TRANSPORT_SEED
    n = args.photons

    tune = pm.Tune(waves_per_cu=args.waves_per_cu, defer=args.defer)

    def one_step(timed):
        res = pm.run(mask, opt, n, seed, timed=timed, tune=tune)
        summ, depth, ws = pm.reduce_async(mask, res)
        return res, summ

    for i in range(args.warmup):
        res, summ = one_step(False)
        torch.cuda.synchronize()
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    walk_ms = []
    steps_total = 0
    t_start = time.perf_counter()
    outs = []
    for i in range(args.steps):
        res, summ = one_step(True)
        walk_ms.append(res.walk_ms)   # waits for this step's walk (events on the run's stream)
        outs.append((res.scalars, summ))
        log(f"step {i}: walk {res.walk_ms:.1f} ms")
    torch.cuda.synchronize()
    t_el = time.perf_counter() - t_start
    ms_per_step = 1e3 * t_el / args.steps
    sc = outs[-1][0].cpu().numpy()
    steps_per_run = int(sc[pm.SCALARS.index("steps")])
    for s, _ in outs:
        assert torch.equal(s, outs[0][0]), "runs are not bitwise identical"
    q = outs[-1][1].cpu().numpy()
    summary = {k: float(q[i]) for i, k in enumerate(pm.SUMMARY)}
    assert summary["closure_exact"] == 1.0
    steps_per_s = steps_per_run * args.steps / t_el
    photons_per_s = n * args.steps / t_el
    walk_avg_ms = float(np.mean(walk_ms))
    achieved_gbs = steps_per_run * BYTES_PER_STEP / (walk_avg_ms * 1e-3) / 1e9
    del res, outs
    # the same workload once through the FP64 reference transport (outside the timed steps)
    r64 = pm.run(mask, opt, n, seed, timed=True, fp64=True, tune=tune)
    s64 = pm.reduce(mask, r64)
    fp64_leg = {"walk_ms": r64.walk_ms, "photon_steps": int(s64["steps_per_photon"] * n),
                "photon_steps_per_s": s64["steps_per_photon"] * n / (r64.walk_ms * 1e-3),
                "walk_time_vs_fp32": r64.walk_ms / walk_avg_ms,
                "relative_difference_vs_fp32": {k: abs(s64[k] - summary[k]) / abs(summary[k])
                                                for k in ("phi3d", "phi1d", "r", "R", "T", "A")}}
    log(f"FP64 transport: walk {r64.walk_ms:.1f} ms ({r64.walk_ms / walk_avg_ms:.2f}x the FP32 walk)")
    del r64
    line = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "photon-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "plain: 256^3 Cahn-wave mask phi=0.70 (lambda 24), mu_s 0.5 mu_a 0.01 g 0.7, "
                               "1e8 photons per step, seed 20260809",
                   "photons_per_step": n, "photon_steps_per_step": steps_per_run, "tallies": "int64 fixed point"},
        "photons_per_s": photons_per_s,
        "mask_h2d": {"bytes": int(mask_np.nbytes), "ms": h2d_ms,
                     "GB_per_s": mask_np.nbytes / (h2d_ms * 1e-3) / 1e9,
                     "note": "uint8 mask, pinned host memory to HBM, once per run, not in the timed steps"},
        "walk_ms_avg": walk_avg_ms,
        "walk_ms_median": float(np.median(walk_ms)),
        "fp64_transport": fp64_leg,
        "roofline": {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved_gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_walk", "algorithmic_bytes_per_step": BYTES_PER_STEP},
        "results": {k: summary[k] for k in ("phi3d", "phi1d", "r", "ratio", "identity_rhs", "R", "T", "A",
                                             "steps_per_photon", "Pw_void_gtL", "mean_void_path")},
    }

    tr = recorded_traffic(n)
    if tr is not None:
        rec, _ = tr
        traffic, line["atomic_request_roof"], line["valu_roof"] = plain_roofs(rec, n, steps_per_run, walk_avg_ms)
        line["roofline"]["traffic"] = traffic

    if not args.no_rows:
        line["rows"] = rows_leg(args, seed, field)
    del field
    if not args.no_paper:
        line["paper_boundary"] = paper_leg(args, seed, mask_np, mask)
    if not args.no_ch:
        line["spinodal_generator"] = ch_leg(args)
    if not args.no_analytics:
        line["analytics"] = analytics_leg(args, seed, mask_np, mask)
    if not args.no_batch:
        line["batched"] = batched_leg(args, seed)
    if not args.no_morph:
        line["morphology_control"] = morphology_leg(args, seed)
    if not args.no_grad:
        line["differentiated"] = grad_leg(args, seed, mask)

    if not args.no_cpu:
        import oracle
        from oracle import estimators as est
        ncpu = len(os.sched_getaffinity(0))
        m = args.cpu_photons
        log(f"oracle: {m} photons on {ncpu} threads")
        t1 = time.perf_counter()
        ref = oracle.run(mask_np, opt.mu_s, opt.mu_a, opt.g, m, seed, nthreads=ncpu)
        t_cpu = time.perf_counter() - t1
        tot = oracle.totals(ref)
        # the same photons on the GPU, for the error against the oracle
        sub = pm.run(mask, opt, m, seed)
        ssum = pm.reduce(mask, sub)
        e = est.estimators(ref["fluence"][0], mask_np, m)
        err = {k: abs(ssum[k] - e[k]) / abs(e[k]) for k in ("phi3d", "phi1d", "r")}
        gsc = sub.scalar_dict()
        for k in ("R", "T", "A"):
            err[k] = abs(gsc[k] - tot[k]) / (m * pm.W1)
        err["steps"] = abs(gsc["steps"] - tot["steps"]) / tot["steps"]
        line["cpu_baseline"] = {"value": tot["steps"] / t_cpu, "unit": "photon-steps/s", "cores": ncpu,
                                "kind": "oracle", "photons_per_s": m / t_cpu,
                                "sample": f"first {m} photon ids of the same workload (same mask, optics, seed), "
                                          f"FP64, {ncpu} threads, {cpu_model()}",
                                "seconds": t_cpu}
        line["oracle_error"] = err
        line["gpu_over_cpu"] = steps_per_s / (tot["steps"] / t_cpu)
        # the same oracle on one host thread, over a smaller sample of the same ids
        m1 = max(1, m // 60)
        t1 = time.perf_counter()
        ref1 = oracle.run(mask_np, opt.mu_s, opt.mu_a, opt.g, m1, seed, nthreads=1, fluence=False)
        t_one = time.perf_counter() - t1
        line["cpu_baseline"]["one_core"] = {"value": oracle.totals(ref1)["steps"] / t_one, "photons": m1,
                                            "seconds": t_one}
    line["paper_context"] = paper_context(line)
    bad = oracle_tolerance_failures(line)
    line["oracle_within_tolerance"] = not bad
    line["oracle_tolerance_failures"] = bad
    print(json.dumps(line), flush=True)
    if bad:
        log("oracle agreement outside tolerance: " + "; ".join(bad))
    # the headline workload's own comparison (3e6 shared photons) must hold
    if any(b.startswith("plain.") for b in bad):
        sys.exit(3)


def paper_context(line) -> dict:
    """The paper's <Phi>_3D / <Phi>_1D ratios (abstract; Sec. 3.6, Table 4) beside this run's,
    as context only: the paper's runs use its own Cahn-Hilliard masks, mirrors, Fresnel faces
    and shell optics, name no GPU model and report no throughput."""
    ours = {"plain_model_phi070": line["results"]["ratio"]}
    row = (line.get("rows") or {}).get("M2b_256cube_phi090")
    if row:
        ours["plain_model_phi090"] = row["phi3d"] / row["phi1d"]
    pb = line.get("paper_boundary") or {}
    if "paper_optics" in pb:
        ours["paper_model_paper_optics_phi070"] = pb["paper_optics"]["ratio"]
    return {"ratio_phi3d_over_phi1d": {"paper_phi070": 1.515, "paper_phi090": 1.774, "this_run": ours},
            "paper_hardware": "not stated (the GPU Monte Carlo code MCX through its Python interface)",
            "note": "context only; the synthetic masks and the plain model's boundaries and optics differ"}


def oracle_tolerance_failures(line) -> list:
    """Every oracle comparison in the line against the stated bars: the estimators and
    R/T/A within 0.5 %, steps within 0.1 % (0.2 % for the samples of 1e5 to 1e6
    photons, whose FP32 divergences weigh more)."""
    bad = []

    def check(name, err, steps_tol):
        for k, v in err.items():
            tol = steps_tol if k == "steps" else 5e-3
            if not (v <= tol):
                bad.append(f"{name}.{k} = {v:.2e} > {tol:.0e}")

    if "oracle_error" in line:
        check("plain", line["oracle_error"], 1e-3)
    for name, row in (line.get("rows") or {}).items():
        if row.get("oracle"):
            check(name, row["oracle"]["relative_error"], 2e-3)
    for name, row in (line.get("paper_boundary") or {}).items():
        if isinstance(row, dict) and row.get("oracle"):
            check("paper_" + name, row["oracle"]["relative_error"], 2e-3)
    for name, row in ((line.get("batched") or {}).get("oracle") or {}).items():
        check("batched_" + name, row["relative_error"], 2e-3)
    for name, row in ((line.get("morphology_control") or {}).get("oracle") or {}).items():
        check("morphology_" + name, row["relative_error"], 2e-3)
    return bad


if __name__ == "__main__":
    main()
