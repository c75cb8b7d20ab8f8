#!/usr/bin/env python3
"""Throughput of the truncated-Wigner ensemble hot path on one MI355X.

One timed run = the whole method on the 2D workload (512^2 grid, 256 Wigner
realizations plus the classical field, FP64): Wigner sampling, K leapfrog
steps (drift / Poisson / kick / drift, Sec. "Integrating the equations of
motion") and the ensemble moments including energies. The metric is
realization*cell*steps per second. Prints ONE JSON line on stdout.

Extra objects in the line:
  roofline      the dominant kernel's algorithmic HBM bytes per launch over its
                average duration (HIP events on the launch stream, same timed run)
  cpu_baseline  the CPU FP64 oracle timed on a bounded sample of the workload
  fp32_split    the FP32-split form on the same workload, with its normwise error
                against the FP64 run for each per-cell moment
  adaptive      the same workload with step sizes chosen on the device
  tracers       the same workload with test particles in every field
  resident_1d   the 1D workload (fields resident in one workgroup for all steps)
  diagnostics   tw_moments with every optional output
  kgauss_512sq  the paper's momentum-space Gaussian problem at 512^2 (FP64, device-chosen steps)
  scale_512cube the paper's momentum-space Gaussian problem at 512^3 (FP32)
  batched       the three-size 3D soliton ensemble advanced from one HIP graph
  surrogate     the reduced FNO surrogate study
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "realization·cell·steps/s"
# the headline: throughput, with the dominant kernel's share of the HBM
# roofline (`roofline`) and the FP32 and surrogate forms against FP64 at a
# stated error (`fp32_split`, `surrogate`) in the same line
HEADLINE = "realization·cell·steps/s + % HBM roofline; FP32/surrogate vs FP64 at fixed error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(kind, elem, ncell, nfield, n_real):
    """Algorithmic (compulsory) HBM bytes of one launch of a kernel kind: every
    input read once and every output written once."""
    npairs = (nfield + 1) // 2
    f = elem * ncell * nfield      # all fields once
    z = elem * ncell * npairs      # spectral scratch once (one complex field per pair)
    return {
        "pass_drift": 2 * f,
        "pass_drift_rho": 2 * f + z,
        "pass_zfwd": 2 * z, "pass_zinv": 2 * z, "pass_zpoisson": 2 * z,
        "pass_kick_drift": z + 2 * f,
        "pass_rho": f + z,
        "pass_kin_sum": f,
        "pass_pot_sum": z + f,
        "pass_slab_drift": 2 * f,
        "pass_slab_drift_rho": 2 * f + z,
        "pass_slab_poisson": 2 * z,
        "pass_slab_kick_drift": z + 2 * f,
        "step1d_resident": 2 * f,
        "sample": 16 * ncell + elem * ncell * n_real,
        "moments": elem * ncell * nfield + 40 * ncell,
    }.get(kind)


def alg_bytes_per_cell_step(precision):
    """Algorithmic HBM bytes of the method per realization*cell*step: the state
    read once and written once (complex128: 32 B; complex64: 16 B)."""
    return 32 if precision == "fp64" else 16


# Kernel kinds that make up the steps (tw_step): everything else in a timed run
# (sampling, moment reductions, energy passes) happens once per run.
STEP_KINDS = ("pass_drift", "pass_drift_rho", "pass_zfwd", "pass_zpoisson", "pass_zinv", "pass_kick_drift",
              "pass_slab_drift", "pass_slab_drift_rho", "pass_slab_poisson", "pass_slab_kick_drift", "step1d_resident",
              "field_mean", "tables")


def roofline_of(prof, precision, elem, ncell, nfield, n_real, steps_timed, step_prof=None, ms_per_step=None):
    """Roofline object of a timed run.

    achieved: the algorithmic bytes one launch of the dominant kernel stands
    for (alg_bytes_per_cell_step x the nfield*ncell cells of one step, which
    is what one launch of a step pass covers) over that kernel's average
    launch duration; frac = achieved / peak. The kernel's own compulsory bytes
    (its inputs read once, outputs written once) are reported beside it
    (kernel_gbs, kernel_frac), and, from a profiled call of the steps alone
    (step_prof), the bytes all step passes move per realization*cell*step and
    their ratio to the algorithmic figure (the cost of the pass count)."""
    kind, (launches, total_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_s = total_ms / launches / 1e3
    alg = alg_bytes_per_cell_step(precision) * nfield * ncell
    own = pass_bytes(kind, elem, ncell, nfield, n_real)
    achieved = alg / avg_s / 1e9
    r = {"bound": "hbm", "kernel": kind, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": None,
         "alg_bytes_per_launch": alg, "alg_bytes_per_cell_step": alg_bytes_per_cell_step(precision),
         "avg_launch_ms": avg_s * 1e3, "launches": launches,
         "kernel_bytes_per_launch": own,
         "kernel_gbs": (own / avg_s / 1e9) if own else None,
         "kernel_frac": (own / avg_s / 1e9 / HBM_PEAK_GBS) if own else None}
    if ms_per_step:
        r["step_frac"] = alg / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS
    if step_prof:
        steps = step_prof["steps"]
        tot_b, tot_ms = 0.0, 0.0
        for k, (nl, ms) in step_prof["prof"].items():
            if k not in STEP_KINDS:
                continue
            tot_ms += ms
            b = pass_bytes(k, elem, ncell, nfield, n_real)
            if b:
                tot_b += nl * b
        per_cs = tot_b / (steps * nfield * ncell)
        r["step_kernel_ms"] = tot_ms / steps
        r["step_kernels_frac"] = alg / (tot_ms / steps * 1e-3) / 1e9 / HBM_PEAK_GBS
        r["pass_bytes_per_cell_step"] = per_cs
        r["pass_bytes_ratio"] = per_cs / alg_bytes_per_cell_step(precision)
    return r


def measured_traffic(kind, precision, workload):
    """HBM bytes per launch of `kind` from the committed rocprofv3 counter summary
    (profiles/traffic_<kind>_<workload>_<precision>.json), or None if there is
    none or the kernel sources changed since the counters were taken."""
    from paper_2310_07119_amd import traffic
    fn = os.path.join(ROOT, "profiles", f"traffic_{kind}_{workload}_{precision}.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as f:
        d = json.load(f)
    if d.get("source_digest") != traffic.source_digest():
        return None
    return d.get("traffic_bytes_per_launch")


def stream_bandwidth():
    """Best read+write streaming rate this device reaches in a plain kernel
    (torch.add over 1 GiB in and 1 GiB out), GB/s: the practical ceiling next
    to the 8 TB/s published peak."""
    import torch
    n = 1 << 28
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(100):
        torch.add(x, 1.0, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(100):
        torch.add(x, 1.0, out=y)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 100
    del x, y
    torch.cuda.empty_cache()
    return 2 * 4 * n / (ms * 1e-3) / 1e9


def run_gpu(wl, precision, steps, warmup, seed=20231007):
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision=precision)
    dev = torch.device("cuda:0")
    plan = Plan(p)
    variant = plan.autotune()
    cl64 = torch.from_numpy(inputs.initial_field(wl["name"])).to(dev)
    psi = plan.empty_ensemble(dev)
    clt = torch.empty(p.shape, dtype=p.cdtype, device=dev)
    dt = wl["dt"]

    def one_run(k):
        plan.sample(cl64, seed, 0, out=psi)
        clt.copy_(cl64.to(p.cdtype))
        plan.step(psi, k, dt, clt)
        return plan.moments(psi, clt, energy=True)

    if warmup > 0:
        one_run(warmup)
    torch.cuda.synchronize()
    plan.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mom = one_run(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile()
    elapsed = t1 - t0
    # the steps alone, profiled once more outside the timed region: bytes and
    # kernel time per step without sampling and moments
    plan.step(psi, steps, dt, clt)
    torch.cuda.synchronize()
    step_prof = {"steps": steps, "prof": plan.profile()}
    plan.set_profiling(False)
    work = p.n_real * p.ncell * steps
    res = dict(value=work / elapsed, ms_per_step=1e3 * elapsed / steps, elapsed_s=elapsed, prof=prof,
               mom={k: (v.cpu() if torch.is_tensor(v) else v) for k, v in mom.items()},
               problem=p)
    elem = 16 if precision == "fp64" else 8
    nfield = p.n_real + 1
    rl = roofline_of(prof, precision, elem, p.ncell, nfield, p.n_real, steps, step_prof, res["ms_per_step"])
    traffic = measured_traffic(rl["kernel"], precision, wl["name"])
    rl["traffic"] = traffic
    # compulsory bytes of the kernel / bytes the counters saw it move (1 = no wasted traffic)
    rl["pass_efficiency"] = (rl["kernel_bytes_per_launch"] / traffic) if (rl["kernel_bytes_per_launch"] and traffic) else None
    res["roofline"] = rl
    res["kernel_ms"] = {k: round(v[1], 3) for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1])}
    res["strided_variant"] = variant
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()
    return res


def run_adaptive(wl, precision, steps, warmup, seed=20231007, courant=0.5):
    """The same workload advanced by tw_step_adaptive (step sizes chosen on the
    device from max|V| and the kinetic bound, no host synchronisation), timed
    like the fixed-step run; reports the step sizes it chose."""
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision=precision)
    plan = Plan(p)
    plan.autotune()
    cl = torch.from_numpy(inputs.initial_field(wl["name"])).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    dt_max = 10.0 * wl["dt"]
    if warmup > 0:
        plan.step_adaptive(psi, warmup, dt_max, courant, clt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dts = plan.step_adaptive(psi, steps, dt_max, courant, clt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = dts.cpu()
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()
    return {"value": p.n_real * p.ncell * steps / el, "unit": METRIC, "ms_per_step": 1e3 * el / steps,
            "courant": courant, "dt_max": dt_max, "dt_min_chosen": float(d.min()), "dt_max_chosen": float(d.max()),
            "simulated_time": float(d.sum()), "timed": "tw_step_adaptive only (no sampling or moments)"}


def run_kgauss_2d(steps, seed=5, courant=0.5):
    """The paper's 2D momentum-space Gaussian at its full size (512^2, 64
    realizations + the classical field, FP64, physical units) with step sizes
    chosen on the device (dt_max 10 Myr): sampling, steps, moments."""
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    wl = dict(inputs.WORKLOADS["2d_n512_kgauss"])
    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision="fp64")
    plan = Plan(p)
    plan.autotune()
    cl = torch.from_numpy(inputs.initial_field("2d_n512_kgauss")).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.clone()
    plan.step_adaptive(psi, 2, wl["dt"], courant, clt)      # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    psi = plan.sample(cl, seed, out=psi)
    clt.copy_(cl)
    dts = plan.step_adaptive(psi, steps, wl["dt"], courant, clt)
    m = plan.moments(psi, clt, energy=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d = dts.cpu()
    out = {"workload": "2d_n512_kgauss", "grid": list(p.n), "n_real": p.n_real, "precision": "fp64",
           "value": p.n_real * p.ncell * steps / el, "unit": METRIC, "ms_per_step": 1e3 * el / steps,
           "steps": steps, "dt_myr_first": float(d[0]), "dt_myr_last": float(d[-1]),
           "simulated_myr": float(d.sum()), "Q_raw": m["Q_raw"], "norm_mean": m["norm_mean"],
           "timed": "tw_sample + tw_step_adaptive + tw_moments (with energies)"}
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()
    return out


def run_tracers(wl, precision, steps, warmup, ntracer=64, seed=20231007):
    """The same workload with ntracer test particles per field pushed in every
    field's own potential (tw_step_tracers); reports the step time and the
    particles' spread over the realizations at the end."""
    import numpy as np
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision=precision)
    plan = Plan(p)
    plan.autotune()
    cl = torch.from_numpy(inputs.initial_field(wl["name"])).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    D = len(p.n)
    rng = np.random.default_rng(seed)
    tr0 = np.zeros((p.n_real + 1, ntracer, 2 * D))
    tr0[:, :, :D] = rng.uniform(0.0, 1.0, (1, ntracer, D)) * np.array(p.box)   # same start in every field
    tr = torch.from_numpy(tr0).cuda()
    if warmup > 0:
        plan.step_tracers(psi, warmup, wl["dt"], tr, clt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step_tracers(psi, steps, wl["dt"], tr, clt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    spread = plan.tracer_spread(tr).cpu().numpy()
    plan.close()
    del psi, clt, tr
    torch.cuda.empty_cache()
    prod = np.sqrt(spread[:, :D] * spread[:, D:])
    return {"value": p.n_real * p.ncell * steps / el, "unit": METRIC, "ms_per_step": 1e3 * el / steps,
            "tracers_per_field": ntracer, "median_dx_dp": float(np.median(prod)),
            "timed": "tw_step_tracers only"}


def run_1d(seed=0):
    """The 1D workload (256 points, 64 realizations + classical field, 1000
    steps, FP64): every field stays resident in one workgroup for all steps, so
    HBM is touched only at the ends; reported with the FP64 arithmetic rate it
    implies (about 230 FP64 operations per cell and step: four 256-point
    transforms at 5 n log2 n / n, the drift and kick factors, density, Green's
    function)."""
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    wl = dict(inputs.WORKLOADS["1d_n256"])
    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision="fp64")
    plan = Plan(p)
    cl = torch.from_numpy(inputs.initial_field("1d_n256")).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.clone()
    plan.step(psi, 10, wl["dt"], clt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.step(psi, wl["nsteps"], wl["dt"], clt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    plan.close()
    rate = p.n_real * p.ncell * wl["nsteps"] / el
    flops = 4 * 5 * 8 + 70   # per cell and step
    return {"workload": "1d_n256", "value": rate, "unit": METRIC, "seconds": el, "steps": wl["nsteps"],
            "fp64_tflops_estimate": rate * flops / 1e12, "fp64_peak_tflops": 78.6}


def run_diagnostics(wl, precision, seed=20231007, reps=3):
    """tw_moments with every optional output (energies, per-mode occupations,
    amplitude and phase spread) on the sampled workload ensemble."""
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision=precision)
    plan = Plan(p)
    plan.autotune()
    cl = torch.from_numpy(inputs.initial_field(wl["name"])).cuda()
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    plan.moments(psi, clt, energy=True, modes=True, decoherence=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        m = plan.moments(psi, clt, energy=True, modes=True, decoherence=True)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    plan.close()
    del psi, clt
    torch.cuda.empty_cache()
    return {"ms_per_call": 1e3 * el, "Q_raw": m["Q_raw"], "Var_A": m["Var_A"], "Var_phi": m["Var_phi"],
            "timed": "tw_moments with energies, mode occupations and amplitude/phase spread"}


def run_scale(steps, seed=5):
    """The paper's momentum-space Gaussian test problem at 512^3 (FP32 split,
    32 realizations + classical field, about 50 GiB of HBM): sampling, steps
    with device-chosen sizes, moments."""
    import torch
    from paper_2310_07119_amd import Plan, Problem, inputs

    wl = dict(inputs.WORKLOADS["3d_n512_kgauss"])
    p = Problem(n=wl["n"], box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                n_tot=wl["n_tot"], n_real=wl["n_real"], precision="fp32")
    t_ic = time.perf_counter()
    cl = torch.from_numpy(inputs.initial_field("3d_n512_kgauss")).cuda()
    t_ic = time.perf_counter() - t_ic
    plan = Plan(p)
    plan.autotune()
    psi = plan.sample(cl, seed)
    clt = cl.to(p.cdtype).clone()
    plan.step_adaptive(psi, 1, wl["dt"], 0.5, clt)      # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dts = plan.step_adaptive(psi, steps, wl["dt"], 0.5, clt)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m = plan.moments(psi, clt, energy=True)
    free, total = torch.cuda.mem_get_info()
    out = {"workload": "3d_n512_kgauss", "grid": list(p.n), "n_real": p.n_real, "precision": "fp32",
           "value": p.n_real * p.ncell * steps / el, "unit": METRIC, "ms_per_step": 1e3 * el / steps,
           "dt_myr": float(dts[0]), "norm_mean": m["norm_mean"], "hbm_in_use_gib": round((total - free) / 2 ** 30, 1),
           "host_ic_seconds": round(t_ic, 1)}
    plan.close()
    del psi, clt, cl
    torch.cuda.empty_cache()
    return out


def run_batched(steps, warmup, seed=7):
    """The three-size 3D soliton ensemble (FP32 split) advanced as one batch:
    every pass is one grouped launch over all classes and the K steps are one
    HIP graph launch. Also times the same classes advanced one plan at a time."""
    import torch
    from paper_2310_07119_amd import Batch, Plan, Problem, inputs

    wl = inputs.WORKLOADS["3d_batched_soliton"]
    probs = [Problem(n=n, box=wl["box"], hbar_m=wl["hbar_m"], G=wl["G"], m_tot=wl["m_tot"],
                     n_tot=wl["occupation"] * n[0] * n[1] * n[2], n_real=wl["n_real"], precision="fp32")
             for n in wl["classes"]]
    batch = Batch(probs)
    variant, mode = batch.autotune()
    psis = []
    for p, plan in zip(probs, batch.plans):
        cl = torch.from_numpy(inputs.soliton_3d(p.n, p.box, core=0.1)).cuda()
        psis.append(plan.sample(cl, seed))
    dt = wl["dt"]
    work = sum(p.n_real * p.ncell for p in probs) * steps
    batch.step(psis, steps, dt)          # capture + warm
    for _ in range(max(warmup, 0)):
        batch.step(psis, steps, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.step(psis, steps, dt)          # one graph launch
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    singles = [Plan(p) for p in probs]
    for pl in singles:
        pl.autotune()
    for pl, x in zip(singles, psis):
        pl.step(x, steps, dt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, x in zip(singles, psis):
        pl.step(x, steps, dt)
    torch.cuda.synchronize()
    el1 = time.perf_counter() - t0
    # error against the plain FP64 path: the same draws (the FP32 state is the
    # FP64 draw rounded), advanced by the batch in FP32 and by one FP64 plan
    # per class, moments compared normwise per class
    err = []
    for c, p in enumerate(probs):
        cl = torch.from_numpy(inputs.soliton_3d(p.n, p.box, core=0.1)).cuda()
        psis[c] = batch.plans[c].sample(cl, seed)
    batch.step(psis, steps, dt)
    p64s = [Problem(n=p.n, box=p.box, hbar_m=p.hbar_m, G=p.G, m_tot=p.m_tot, n_tot=p.n_tot, n_real=p.n_real,
                    precision="fp64") for p in probs]
    for c, (p, p64) in enumerate(zip(probs, p64s)):
        m32 = batch.plans[c].moments(psis[c], energy=True)
        plan64 = Plan(p64)
        cl = torch.from_numpy(inputs.soliton_3d(p.n, p.box, core=0.1)).cuda()
        x64 = plan64.sample(cl, seed)
        plan64.step(x64, steps, dt)
        m64 = plan64.moments(x64, energy=True)
        err.append({"class": list(p.n), **{k: rel(m32[k], m64[k]) for k in ("mean_psi", "mean_rho", "var_rho", "norm",
                                                                              "energy")}})
        plan64.close()
        del x64
    torch.cuda.empty_cache()
    out = {"workload": "3d_batched_soliton", "classes": [list(p.n) for p in probs],
           "err_vs_fp64": err,
           "n_real_per_class": wl["n_real"], "precision": "fp32", "steps": steps,
           "value": work / el, "unit": METRIC, "ms_per_step": 1e3 * el / steps,
           "unbatched_value": work / el1, "speedup_vs_unbatched": el1 / el, "strided_pass_variant": variant,
           "batch_mode": ["grouped launches", "per-class graph branches"][mode],
           "launch": "one hipGraph launch for all classes and all steps"}
    batch.close()
    for pl in singles:
        pl.close()
    del psis
    torch.cuda.empty_cache()
    return out


def _oracle_steps(args):
    """One copy of the oracle stepping its own ensemble for about budget_s
    seconds (runs in a worker process; numpy only)."""
    n, box, hbar_m, G, m_tot, dt, psi, budget_s = args
    from oracle import twa_oracle as tw
    prob = tw.Problem(tw.Grid(n, box), hbar_m, G, m_tot)
    t0 = time.perf_counter()
    steps = 0
    while True:
        psi = tw.step(prob, psi, dt)
        steps += 1
        if time.perf_counter() - t0 > budget_s and steps >= 2:
            break
    return psi.shape[0] * prob.grid.ncell * steps, steps, time.perf_counter() - t0


def _fno_oracle_times(seed=5):
    """The surrogate's oracle (numpy, BF16 operands emulated) on one 256^2
    field of the surrogate study's shape, one BLAS thread: seconds for a
    forward pass and for a backward pass (which includes its forward)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fno_oracle as fo
    cfg = fo.Config(H=256, W=256, c_in=4, width=32, mx=16, my=16, layers=4, proj=128, c_out=2)
    params = fo.init_params(cfg, seed)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((1, cfg.H, cfg.W, cfg.c_in))
    dy = rng.standard_normal((1, cfg.H, cfg.W, cfg.c_out))
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        fo.forward(cfg, params, x)
        t1 = time.perf_counter()
        fo.backward(cfg, params, x, dy)
        t2 = time.perf_counter()
    return {"forward_s": t1 - t0, "forward_backward_s": t2 - t1, "threads": 1,
            "field": "256x256, 4 input channels, width 32, 4 Fourier layers of 32x16 modes, projection 128"}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def cpu_baseline(wl, budget_s=15.0, n_sample_real=4, seed=20231007, max_workers=16):
    """The oracle as it stands, on a bounded sample: n_sample_real realizations of
    the full grid, as many steps as fit in about budget_s seconds, first in this
    process (one thread: numpy's FFT and elementwise work are single-threaded),
    then as independent copies in one worker process per available core (at
    most max_workers), each stepping its own copy of the sample, which is how
    the ensemble's independent realizations parallelise on a CPU. `value` is
    the all-core rate."""
    import subprocess
    import tempfile

    import numpy as np

    from oracle import twa_oracle as tw
    from paper_2310_07119_amd import inputs

    grid = tw.Grid(wl["n"], wl["box"])
    psi_cl = inputs.initial_field(wl["name"])
    psi = tw.sample(grid, psi_cl, n_sample_real, wl["n_tot"], seed)
    job = (tuple(wl["n"]), tuple(wl["box"]), wl["hbar_m"], wl["G"], wl["m_tot"], wl["dt"], psi, budget_s)
    work1, steps1, el1 = _oracle_steps(job)
    single = work1 / el1
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(max_workers, ncpu))
    allc, steps_w = None, None
    if workers > 1:
        # independent child interpreters (numpy only, no GPU), each stepping its
        # own copy of the sample; killed if they overrun
        with tempfile.TemporaryDirectory() as tmp:
            fn = os.path.join(tmp, "psi.npy")
            np.save(fn, psi)
            code = ("import json, sys; sys.path.insert(0, sys.argv[1]); import numpy as np; "
                    "from bench import _oracle_steps; "
                    "a = json.loads(sys.argv[3]); "
                    "w, st, el = _oracle_steps((tuple(a['n']), tuple(a['box']), a['hbar_m'], a['G'], a['m_tot'], "
                    "a['dt'], np.load(sys.argv[2]), a['budget_s'])); "
                    "print(json.dumps([w, st, el]))")
            spec = json.dumps(dict(n=list(wl["n"]), box=list(wl["box"]), hbar_m=wl["hbar_m"], G=wl["G"],
                                   m_tot=wl["m_tot"], dt=wl["dt"], budget_s=budget_s))
            procs = [subprocess.Popen([sys.executable, "-c", code, ROOT, fn, spec], stdout=subprocess.PIPE,
                                      stderr=subprocess.DEVNULL, text=True) for _ in range(workers)]
            res = []
            try:
                for pr in procs:
                    o, _ = pr.communicate(timeout=4 * budget_s + 120)
                    if pr.returncode == 0:
                        res.append(json.loads(o.strip().splitlines()[-1]))
            except (subprocess.TimeoutExpired, ValueError, IndexError) as e:
                log(f"cpu oracle: worker processes failed ({e}); reporting the single-thread rate")
            finally:
                for pr in procs:
                    if pr.poll() is None:
                        pr.kill()
                        pr.wait()
            if len(res) == workers:
                allc = sum(w / e for w, _, e in res)
                steps_w = min(st for _, st, _ in res)
    fno = _fno_oracle_times()
    model = _cpu_model()
    sample = (f"{n_sample_real} realizations x {steps1} leapfrog steps of the {wl['name']} grid "
              f"{'x'.join(map(str, wl['n']))} (numpy FP64), {el1:.1f} s on one thread")
    if allc is None:
        return {"value": single, "unit": METRIC, "cores": 1, "kind": "oracle", "sample": sample + f"; {model}",
                "nproc": ncpu, "fno_oracle": fno}
    sample += (f"; then {workers} worker processes, each stepping its own copy of the sample (>= {steps_w} "
               f"steps in about {budget_s:.0f} s); {model}")
    return {"value": allc, "unit": METRIC, "cores": workers, "kind": "oracle", "sample": sample,
            "single_thread_value": single, "nproc": ncpu, "fno_oracle": fno}


def rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="2d_n512_pair")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-grf128", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true")
    ap.add_argument("--no-tracers", action="store_true")
    ap.add_argument("--no-diagnostics", action="store_true")
    ap.add_argument("--no-1d", dest="no_1d", action="store_true")
    ap.add_argument("--no-scale", action="store_true")
    ap.add_argument("--no-kgauss", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}): realizations "
              "are independent, so a multi-GPU run is N copies of this one with disjoint realization offsets "
              "and no per-step communication; no multi-GPU figure is produced.", file=sys.stderr)
        sys.exit(2)

    from paper_2310_07119_amd import inputs
    wl = dict(inputs.WORKLOADS[args.workload], name=args.workload)
    log(f"workload {args.workload}: grid {wl['n']}, {wl['n_real']} realizations, {args.precision}, "
        f"{args.steps} timed steps after {args.warmup} warmup")
    stream_gbs = stream_bandwidth()  # first: it also brings the device out of idle before the timed legs
    main_run = run_gpu(wl, args.precision, args.steps, args.warmup)
    log(f"main: {main_run['value']:.4e} {METRIC}, {main_run['ms_per_step']:.3f} ms/step; "
        f"kernels {main_run['kernel_ms']}")
    out = {
        "metric": HEADLINE, "value": main_run["value"], "unit": METRIC, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": main_run["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "grid": list(wl["n"]), "box": list(wl["box"]),
                   "n_real": wl["n_real"], "n_tot": wl["n_tot"], "dt": wl["dt"], "hbar_m": wl["hbar_m"],
                   "G": wl["G"], "m_tot": wl["m_tot"], "precision": args.precision,
                   "timed": "tw_sample + K tw_step leapfrog steps + tw_moments (with energies)",
                   "classical_field": "evolved alongside, not counted in the work"},
        "roofline": dict(main_run["roofline"], stream_measured_gbs=stream_gbs),
        "kernel_ms": main_run["kernel_ms"],
        "strided_pass_variant": main_run["strided_variant"],
    }
    if not args.no_fp32 and args.precision == "fp64":
        r32 = run_gpu(wl, "fp32", args.steps, args.warmup)
        m64, m32 = main_run["mom"], r32["mom"]
        out["fp32_split"] = {
            "value": r32["value"], "ms_per_step": r32["ms_per_step"], "speedup": r32["value"] / main_run["value"],
            "roofline_frac": r32["roofline"]["frac"], "kernel": r32["roofline"]["kernel"],
            "step_frac": r32["roofline"].get("step_frac"), "pass_bytes_ratio": r32["roofline"].get("pass_bytes_ratio"),
            "strided_pass_variant": r32["strided_variant"],
            "err_vs_fp64": {k: rel(m32[k], m64[k]) for k in ("mean_psi", "mean_rho", "var_rho", "norm", "energy")},
        }
        log(f"fp32: {r32['value']:.4e}, errors {out['fp32_split']['err_vs_fp64']}")
    if not args.no_adaptive:
        out["adaptive"] = run_adaptive(wl, args.precision, args.steps, args.warmup)
        ad = out["adaptive"]
        ad["fixed_step_ms_per_step"] = main_run["ms_per_step"]
        # simulated time per wall second against the fixed-step run's
        ad["speedup_per_simulated_time"] = (ad["simulated_time"] / (args.steps * ad["ms_per_step"])) / (
            wl["dt"] / main_run["ms_per_step"])
        log(f"adaptive: {out['adaptive']}")
    if not args.no_tracers:
        out["tracers"] = run_tracers(wl, args.precision, args.steps, args.warmup)
        out["tracers"]["fixed_step_ms_per_step"] = main_run["ms_per_step"]
        log(f"tracers: {out['tracers']}")
    if not args.no_1d:
        out["resident_1d"] = run_1d()
        log(f"1d: {out['resident_1d']}")
    if not args.no_diagnostics:
        out["diagnostics"] = run_diagnostics(wl, args.precision)
        log(f"diagnostics: {out['diagnostics']}")
    if not args.no_kgauss:
        out["kgauss_512sq"] = run_kgauss_2d(args.steps)
        log(f"kgauss 512^2: {out['kgauss_512sq']}")
    if not args.no_scale:
        out["scale_512cube"] = run_scale(max(args.steps // 5, 2))
        log(f"scale: {out['scale_512cube']}")
    if not args.no_grf128:
        # one 3D plan: the 128^3 Gaussian-random-field ensemble, FP32 split
        w3 = dict(inputs.WORKLOADS["3d_n128_grf"], name="3d_n128_grf")
        r3 = run_gpu(w3, "fp32", max(args.steps // 2, 5), 2)
        out["grf_128cube"] = {"workload": "3d_n128_grf", "grid": list(w3["n"]), "n_real": w3["n_real"],
                              "precision": "fp32", "value": r3["value"], "unit": METRIC,
                              "ms_per_step": r3["ms_per_step"], "roofline": r3["roofline"],
                              "kernel_ms": r3["kernel_ms"], "strided_pass_variant": r3["strided_variant"],
                              "timed": "tw_sample + K tw_step leapfrog steps + tw_moments (with energies)"}
        log(f"grf_128cube: {out['grf_128cube']}")
    if not args.no_batched:
        out["batched"] = run_batched(max(args.steps // 2, 1), 1)
        log(f"batched: {out['batched']}")
    if not args.no_surrogate:
        from paper_2310_07119_amd import surrogate
        spec = surrogate.DatasetSpec(n=(256, 256), n_real=128, steps=100, dt=1e-4, n_tot=1e6)
        sres = surrogate.gain_study(spec, n_train=160, n_test=8, epochs=4, batch=8, ref_real=1024, seed=2023)
        sres["note"] = ("reduced study (160 training ensembles, 4 epochs); the full one is "
                        "python -m paper_2310_07119_amd.surrogate --full")
        out["surrogate"] = sres
        log(f"surrogate: {sres}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
        log(f"cpu oracle: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
