"""Benchmark of the Smolyak H|psi> hot path on one MI355X.

Default workload: the (D, L) = (12, 6) coupled-anharmonic Hamiltonian
(omega ~ U(0.5, 2), c ~ U(-0.05, 0.05), k ~ U(-0.02, 0.02), seeded; 18 564
terms, N_cs = 369 305), a displaced-Gaussian wave packet propagated by 500
Chebyshev steps of dt = 0.05 in the precision the mixed-precision autotuner
picks at the 1e-6 bar, with its error against the plain FP64 propagation
after every step.  One benchmark "step" is one Chebyshev time step: K-1
applications of H_S (term sweep + fixed-order reduce with the recurrence
fused into it) over the whole term set.

Prints ONE JSON line: applies/s (value) with the FP64 rate beside it,
grid-points/s (literal and active counts), p50/p99 latency of a single
apply, the dominant kernel's roofline (term sweep: FLOP and HBM fractions),
and the CPU oracle's rate on a bounded sample of the same operator.  The
extra sections cover the (6, 6) FP64 trajectory, the other propagators, 64
batched instances and the serving stream, each mixed against FP64.

`--apply-only N` runs N applies of the workload and exits (the command the
rocprofv3 summaries under profiles/ are taken from).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2 x 2.4 GHz (vector = matrix)
HBM_PEAK_GBS = 8000.0
TOL_MIXED = 1e-6
# Sources whose change invalidates recorded HBM counters of the sweep kernel.
KERNEL_SOURCES = ["paper_2111_13655_amd/csrc/sg_sweep.hip", "paper_2111_13655_amd/csrc/sg_internal.h",
                  "paper_2111_13655_amd/csrc/sg_plan.cpp", "paper_2111_13655_amd/csrc/sg_terms.cpp"]

WORKLOADS = {
    "d12_l6": dict(D=12, L=6, dt=0.05, steps=500, check_every=100, cfg="config2",
                   desc="smolyak H|psi> D=12 L=6 coupled anharmonic (18564 terms, N_cs=369305), "
                        "Chebyshev dt=0.05, mixed precision tuned at 1e-6 vs FP64"),
    "d6_l6": dict(D=6, L=6, dt=0.05, steps=1000, check_every=100, cfg="config1",
                  desc="smolyak H|psi> D=6 L=6 coupled anharmonic, Chebyshev dt=0.05, FP64"),
    "d2_l4": dict(D=2, L=4, dt=0.1, steps=100, check_every=10, cfg="config0",
                  desc="smolyak H|psi> D=2 L=4 coupled anharmonic, Chebyshev dt=0.1, FP64"),
    # general tabulated potential (profiling only: --apply-only)
    "tab_d8_l6": dict(D=8, L=6, dt=0.05, steps=100, check_every=10, cfg="tabulated_d8_l6",
                      desc="general potential tabulated on the term grids, D=8, L=6, FP64"),
    # two-state model (profiling only: --apply-only)
    "vib_d12_l5": dict(D=12, L=5, dt=0.05, steps=100, check_every=10, cfg="vibronic_pyrazine",
                       desc="two-state pyrazine form, 12 modes, L=5, FP64"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def instance_for(name):
    import sg_inputs
    return getattr(sg_inputs, WORKLOADS[name]["cfg"])()


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def recorded_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summaries
    under profiles/ (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when
    none was recorded for this workload or the kernel sources changed since."""
    import glob
    want = kernel_sources_sha256()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-data:"):
                    continue
                kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
                if kv.get("workload") == workload and kv.get("kernel") == kernel:
                    if kv.get("sources_sha256") != want:
                        return None
                    return float(kv["bytes_per_launch"])
    return None


def literal_grid_points(levels, nq_a=2, nq_b=2):
    return int(np.prod([nq_a + nq_b * int(l) for l in levels]))


def cpu_baseline(inst, budget_s: float):
    """The FP64 oracle's literal Alg. 1 (test infrastructure) on a bounded
    sample: whole applies when they fit the budget, else a seeded random sample
    of terms, extrapolated to the whole apply by the literal grid-point share
    of the sampled terms."""
    from oracle.action import Oracle
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    cores = len(os.sched_getaffinity(0))
    O = Oracle(inst)
    S = O.S
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(S.n_cs) + 1j * rng.standard_normal(S.n_cs)
    pts = np.array([literal_grid_points(l, inst.nq_A, inst.nq_B) for l in S.terms], dtype=np.float64)
    total_pts = float(pts.sum())
    order = rng.permutation(S.n_terms)
    done_pts, n_terms_done = 0.0, 0
    t0 = time.perf_counter()
    for t in order:
        O.apply_literal(psi, terms=[int(t)])
        done_pts += pts[t]
        n_terms_done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    apply_s = dt * total_pts / done_pts
    if n_terms_done == S.n_terms:
        sample = f"one whole FP64 apply of the literal per-term oracle (Alg. 1), {dt:.1f} s"
    else:
        sample = (f"{n_terms_done} of {S.n_terms} terms (seeded random order) of one FP64 apply of "
                  f"the literal per-term oracle (Alg. 1) in {dt:.1f} s, "
                  f"{100 * done_pts / total_pts:.2f}% of its literal grid points; "
                  f"extrapolated to {apply_s:.0f} s per apply by that share")
    return {"value": 1.0 / apply_s, "unit": "applies/s", "cores": cores, "kind": "oracle",
            "sample": sample, "blas_threads": int(blas_threads),
            "grid_pts_per_s_literal": total_pts / apply_s,
            "note": "single-threaded NumPy per term; host affinity as 'cores'"}


def _rel(a, b):
    import torch
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def tuned_threshold(sg, P, psi):
    """The mixed-precision autotuner at the 1e-6 bar on the workload's own
    initial state: the fastest FP32 share whose error against the FP64 apply
    stays below half the bar."""
    thr, err = sg.sg_tune_mixed(P.handle, psi, TOL_MIXED, 3)
    return int(thr), float(err)


def step_errors(sg, P, psi0, dt, steps, lo, hi, threshold):
    """Mixed (at `threshold`) and FP64 propagations side by side from psi0:
    relative distance of the mixed state from the FP64 one after every step."""
    import torch
    sg.sg_set_mixed_threshold(P.handle, threshold)
    a64, a32 = psi0.clone(), psi0.clone()
    errs = []
    for _ in range(steps):
        sg.sg_propagate_chebyshev(P.handle, a64, dt, 1, lo, hi, tol=0.0)
        sg.sg_propagate_chebyshev(P.handle, a32, dt, 1, lo, hi, tol=0.0, precision=sg.SG_MIXED)
        errs.append(_rel(a32, a64))
    return errs


def timed_propagation(sg, P, psi0, dt, steps, warmup, lo, hi, prec, check_every):
    import torch
    psi = psi0.clone()
    if warmup > 0:
        sg.sg_propagate_chebyshev(P.handle, psi, dt, warmup, lo, hi, tol=1e-6, precision=prec,
                                  check_every=check_every)
    psi = psi0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, stats, _, _ = sg.sg_propagate_chebyshev(P.handle, psi, dt, steps, lo, hi, tol=1e-6,
                                                    precision=prec, check_every=check_every)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, status, stats, psi


def kernel_times(sg, P, psi0, dt, steps, lo, hi, prec, check_every):
    """Average sweep and reduce durations from HIP events attached to every
    dispatch of `steps` Chebyshev steps, on the stream they are launched on."""
    psi = psi0.clone()
    sg.sg_set_timing(P.handle, True)
    sg.sg_propagate_chebyshev(P.handle, psi, dt, steps, lo, hi, tol=1e-6, precision=prec,
                              check_every=check_every)
    tim = sg.sg_get_timing(P.handle)
    sg.sg_set_timing(P.handle, False)
    return (tim["sweep_ms"] / max(tim["sweep_launches"], 1) * 1e-3,
            tim["reduce_ms"] / max(tim["reduce_launches"], 1) * 1e-3, tim)


def apply_latency(sg, P, x, prec, samples):
    import torch
    y = torch.empty_like(x)
    for _ in range(min(50, samples)):
        P.apply(x, y, prec)
    torch.cuda.synchronize()
    lat = []
    for _ in range(samples):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        P.apply(x, y, prec)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e3)
    lat = np.array(lat)
    return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))


def roofline(info, sweep_s, prec_name, workload):
    flops = info["sweep_flops_fp64"]
    nbytes = info["sweep_bytes"]
    tflops = flops / sweep_s / 1e12
    gbs = nbytes / sweep_s / 1e9
    intensity = flops / nbytes
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    # the FP64 contractions run on the vector ALUs (FP64 vector and matrix
    # peaks are equal on this part)
    bound = "alu" if intensity >= ridge else "hbm"
    if bound == "hbm":
        achieved, peak, unit = gbs, HBM_PEAK_GBS, "GB/s"
    else:
        achieved, peak, unit = tflops, FP64_PEAK_TFLOPS, "TFLOP/s"
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak,
            "traffic": recorded_traffic(f"{workload}/{prec_name}", "sweep_kernel<double>"),
            "kernel": "sweep_kernel<double>",
            "flops_per_launch": flops, "bytes_per_launch": nbytes,
            "intensity_flop_per_byte": intensity, "ridge_flop_per_byte": ridge,
            "flop_frac": tflops / FP64_PEAK_TFLOPS, "hbm_frac": gbs / HBM_PEAK_GBS,
            "achieved_tflops": tflops, "achieved_gbs": gbs}


def headline(sg, args, wl, inst):
    import torch
    log(f"[bench] build {args.workload} D={inst.D} L={inst.L}")
    P = sg.Problem.from_instance(inst)
    info = sg.sg_problem_info(P.handle)
    n = P.n_cs
    psi0 = torch.empty(n, dtype=torch.complex128, device="cuda")
    sg.sg_init_gaussian(P.handle, inst.shift, psi0)
    lo, hi = sg.sg_spectral_bounds(P.handle, 40)
    log(f"[bench] N_cs={n} N_st={info['n_terms']} N_s={info['n_s']} bounds=({lo:.3f},{hi:.3f})")
    dt, steps, ce = wl["dt"], args.steps, wl["check_every"]

    if args.precision == "fp64":
        prec, thr, thr_err = sg.SG_FP64, 0, 0.0
    else:
        thr, thr_err = tuned_threshold(sg, P, psi0)
        prec = sg.SG_MIXED
        log(f"[bench] mixed threshold {thr} (error {thr_err:.2e} on the initial state)")
    prec_name = "fp64" if prec == sg.SG_FP64 else "mixed"

    el, status, stats, _ = timed_propagation(sg, P, psi0, dt, steps, args.warmup, lo, hi, prec, ce)
    applies = stats["applies"]
    log(f"[bench] timed {steps} steps ({prec_name}): {el:.3f} s, {applies} applies, status {status}")
    out_fp64 = None
    if prec != sg.SG_FP64:
        el64, st64, stats64, _ = timed_propagation(sg, P, psi0, dt, steps, 0, lo, hi,
                                                   sg.SG_FP64, ce)
        out_fp64 = {"applies_per_s": stats64["applies"] / el64, "seconds": el64,
                    "status": int(st64)}
        log(f"[bench] fp64 leg: {el64:.3f} s")
    sweep_s, reduce_s, tim = kernel_times(sg, P, psi0, dt, steps, lo, hi, prec, ce)
    log(f"[bench] sweep avg {sweep_s * 1e6:.2f} us, reduce avg {reduce_s * 1e6:.2f} us")
    p50, p99 = apply_latency(sg, P, psi0, prec, args.latency_samples)
    # sweep durations of the FP64 kernel for the roofline (the tuned path may
    # mix FP32 launches in)
    if prec != sg.SG_FP64:
        sweep64_s, reduce64_s, _ = kernel_times(sg, P, psi0, dt, min(steps, 100), lo, hi,
                                                sg.SG_FP64, ce)
    else:
        sweep64_s, reduce64_s = sweep_s, reduce_s
    value = applies / el
    res = {
        "metric": "H|psi> applies/s and grid-pts/s vs plain FP64 at 1e-6 rel err; p50/p99 latency",
        "value": value,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el / max(steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if (prec == sg.SG_FP64 or thr == 0) else "f32+f64",
        "data": "synthetic (seeded coupled-anharmonic Hamiltonian, displaced Gaussian)",
        "config": {"workload": wl["desc"], "D": inst.D, "L": inst.L, "dt": dt,
                   "precision": prec_name, "mixed_threshold": thr, "n_terms": info["n_terms"],
                   "n_cs": n, "n_s": info["n_s"], "chebyshev_terms": stats["cheb_terms"],
                   "check_every": ce, "parallelism": "single GPU",
                   "operator_form": ("split" if (prec == sg.SG_MIXED or info["fp64_split"])
                                     else "grid_kinetic")},
        "grid_pts_per_s_literal": value * info["grid_literal"],
        "grid_pts_per_s_active": value * info["grid_active"],
        "latency_us_p50": p50,
        "latency_us_p99": p99,
        "norm_drift": stats["max_norm_drift"],
        "energy_drift": stats["max_energy_drift"],
        "status": int(status),
        "kernel_avg_us": {"term_sweep": sweep_s * 1e6, "reduce": reduce_s * 1e6,
                          "term_sweep_fp64": sweep64_s * 1e6, "reduce_fp64": reduce64_s * 1e6},
        "roofline": roofline(info, sweep64_s, "fp64", args.workload),
    }
    if prec != sg.SG_FP64:
        res["mixed_vs_fp64"] = {
            "threshold": thr, "apply_rel_err_initial_state": thr_err, "tol": TOL_MIXED,
            "fp64": out_fp64, "mixed_applies_per_s": value,
            "speedup": value / out_fp64["applies_per_s"]}
        if not args.no_error_curve:
            log("[bench] per-step error vs FP64 (tuned threshold)")
            errs = step_errors(sg, P, psi0, dt, steps, lo, hi, thr)
            res["mixed_vs_fp64"]["propagation_rel_err_per_step"] = errs
            res["mixed_vs_fp64"]["propagation_max_rel_err"] = max(errs) if errs else 0.0
            if thr < 1 and args.forced_curve_steps > 0:
                # what FP32 terms would cost: every |D_l| = 1 term in FP32
                log("[bench] per-step error vs FP64 with every |D_l| = 1 term in FP32")
                e1 = step_errors(sg, P, psi0, dt, args.forced_curve_steps, lo, hi, 1)
                x1 = psi0.clone()
                y1 = torch.empty_like(x1)
                y64 = torch.empty_like(x1)
                P.apply(x1, y1, sg.SG_MIXED)
                P.apply(x1, y64, sg.SG_FP64)
                sg.sg_set_mixed_threshold(P.handle, thr)
                res["mixed_vs_fp64"]["threshold_1"] = {
                    "apply_rel_err_initial_state": _rel(y1, y64),
                    "propagation_rel_err_per_step": e1}
    P.close()
    return res


def d6l6_leg(sg, steps=1000):
    """(D, L) = (6, 6), FP64, 1000 Chebyshev steps of dt = 0.05 with norm and
    energy checked every 100 steps."""
    import torch
    import sg_inputs
    inst = sg_inputs.config1()
    with sg.Problem.from_instance(inst) as P:
        psi0 = torch.empty(P.n_cs, dtype=torch.complex128, device="cuda")
        sg.sg_init_gaussian(P.handle, inst.shift, psi0)
        lo, hi = sg.sg_spectral_bounds(P.handle, 40)
        el, status, stats, _ = timed_propagation(sg, P, psi0, 0.05, steps, 20, lo, hi,
                                                 sg.SG_FP64, 100)
        sweep_s, reduce_s, _ = kernel_times(sg, P, psi0, 0.05, 100, lo, hi, sg.SG_FP64, 100)
        p50, p99 = apply_latency(sg, P, psi0, sg.SG_FP64, 1000)
        info = sg.sg_problem_info(P.handle)
    return {"workload": "D=6 L=6, FP64, 1000 steps of dt=0.05, checks every 100",
            "applies_per_s": stats["applies"] / el, "status": int(status),
            "norm_drift": stats["max_norm_drift"], "energy_drift": stats["max_energy_drift"],
            "kernel_avg_us": {"term_sweep": sweep_s * 1e6, "reduce": reduce_s * 1e6},
            "latency_us_p50": p50, "latency_us_p99": p99,
            "sweep_flop_frac": info["sweep_flops_fp64"] / sweep_s / 1e12 / FP64_PEAK_TFLOPS}


def propagators(sg, steps=40, dt=0.05):
    """(D, L) = (6, 6), FP64: the Taylor, Runge-Kutta, short-iterative-Lanczos
    and Bulirsch-Stoer propagators against Chebyshev over the same span, from the
    displaced Gaussian: wall time, applies, and the distance of each final
    state from the Chebyshev one (converged to 1e-16 per step)."""
    import torch
    import sg_inputs
    inst = sg_inputs.config1()
    P = sg.Problem.from_instance(inst)
    n = P.n_cs
    psi0 = torch.empty(n, dtype=torch.complex128, device="cuda")
    sg.sg_init_gaussian(P.handle, inst.shift, psi0)

    def run(fn):
        x = psi0.clone()
        fn(x)   # warm-up, same work
        x = psi0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = fn(x)
        torch.cuda.synchronize()
        return x, time.perf_counter() - t0, st

    lo, hi = sg.sg_spectral_bounds(P.handle, 40)
    ref, t_ref, st_ref = run(lambda x: sg.sg_propagate_chebyshev(P.handle, x, dt, steps,
                                                                 lo, hi)[1])
    out = {"workload": f"D=6 L=6, FP64, {steps} steps of dt={dt}",
           "chebyshev": {"seconds": t_ref, "applies": st_ref["applies"],
                         "applies_per_s": st_ref["applies"] / t_ref}}
    for name, method, order in [("taylor_12", sg.SG_PROP_TAYLOR, 12), ("rk_4", sg.SG_PROP_RK, 4),
                                ("sil_12", sg.SG_PROP_SIL, 12), ("bs_4", sg.SG_PROP_BS, 4)]:
        x, t, st = run(lambda x: sg.sg_propagate(P.handle, x, dt, steps, method, order)[1])
        out[name] = {"seconds": t, "applies": st["applies"], "applies_per_s": st["applies"] / t,
                     "rel_diff_vs_chebyshev": _rel(x, ref)}
    P.close()
    return out


def batched(sg, steps, latency_steps):
    """64 independent instances (D ~ U{4..10}, L ~ U{4..7}), all advanced in
    one launch sequence, mixed and FP64 legs over the same `steps` steps:
    instance-applies/s, p50/p99 of one batched step, and each instance's
    distance from its FP64 result.  The term schedule comes from the batch
    autotuner; each instance's FP32 share from the precision autotuner, asked
    for the 1e-6 bar at the end of the whole propagation (the per-apply error
    budget is the bar divided by the number of applies)."""
    import torch
    import sg_inputs
    insts = sg_inputs.config3()
    probs = [sg.Problem.from_instance(i) for i in insts]
    psi0, lo, hi = [], [], []
    thr = []
    for P, inst in zip(probs, insts):
        x = torch.empty(P.n_cs, dtype=torch.complex128, device="cuda")
        sg.sg_init_gaussian(P.handle, inst.shift, x)
        psi0.append(x)
        a, b = sg.sg_spectral_bounds(P.handle, 40)
        lo.append(a)
        hi.append(b)
        # per instance: the fastest FP32 share whose error on its own initial
        # state stays within the bar spread over the propagation's applies
        K = 14
        t, _ = sg.sg_tune_mixed(P.handle, x, TOL_MIXED / (steps * (K - 1)), 2)
        thr.append(int(t))
    b = sg.sg_batch_create([P.handle for P in probs])
    tuned_g, tuned_ms = sg.sg_batch_tune_schedule(b, psi0, sg.SG_FP64, reps=3)
    dts = [i.meta["dt"] for i in insts]
    legs = {}
    finals = {}
    for name, prec in (("mixed", sg.SG_MIXED), ("fp64", sg.SG_FP64)):
        psis = [x.clone() for x in psi0]
        sg.sg_batch_propagate(b, [x.clone() for x in psi0], dts, 1, lo, hi, tol=1e-6,
                              precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, st = sg.sg_batch_propagate(b, psis, dts, steps, lo, hi, tol=1e-6,
                                           precision=prec, check_every=steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        applies = sum(s["applies"] for s in st)
        grid = sum(P.info["grid_active"] * s["applies"] for P, s in zip(probs, st))
        # per-step latency: single-step calls
        work = [x.clone() for x in psi0]
        lat = []
        for _ in range(latency_steps):
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            sg.sg_batch_propagate(b, work, dts, 1, lo, hi, tol=1e-6, precision=prec)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - s0)
        legs[name] = {"status": int(status), "seconds": el,
                      "instance_applies_per_s": applies / el,
                      "grid_pts_per_s_active": grid / el,
                      "ms_per_batched_step": el / steps * 1e3,
                      "step_latency_ms_p50": float(np.percentile(lat, 50)) * 1e3,
                      "step_latency_ms_p99": float(np.percentile(lat, 99)) * 1e3}
        finals[name] = psis
    errs = [_rel(a, b_) for a, b_ in zip(finals["mixed"], finals["fp64"])]
    sg.sg_batch_free(b)
    for P in probs:
        P.close()
    return {"workload": "64 instances, D ~ U{4..10}, L ~ U{4..7}, dt = 0.05",
            "steps": steps, "mixed": legs["mixed"], "fp64": legs["fp64"],
            "schedule_block_min_grid": tuned_g, "schedule_tuned_apply_ms": tuned_ms,
            "speedup_mixed_vs_fp64": legs["fp64"]["seconds"] / legs["mixed"]["seconds"],
            "mixed_thresholds": thr,
            "instances_with_fp32_terms": int(sum(t > 0 for t in thr)),
            "final_state_rel_err_vs_fp64_max": max(errs),
            "final_state_rel_err_vs_fp64_p50": float(np.percentile(errs, 50)),
            "final_state_rel_err_vs_fp64": errs}


def serve_leg(sg, reqs, precision, mixed_threshold):
    """Submits the requests at their arrival times (relative to the start of
    the leg) and waits for all of them; returns latencies, final states and
    throughput."""
    srv = sg.sg_serve_create(max_slots=64, precision=precision, check_every=100, tol=1e-6,
                             mixed_threshold=mixed_threshold, compile_threads=8)
    tickets = []
    t0 = time.perf_counter()
    for r in reqs:
        now = time.perf_counter() - t0
        if r["arrival_s"] > now:
            time.sleep(r["arrival_s"] - now)
        inst = r["inst"]
        tickets.append((sg.sg_serve_submit(srv, inst.D, r["L"], inst.omega, inst.c, inst.k,
                                           inst.shift, 0.05, r["steps"]), r["n_cs"]))
    lat, applies, ok, statuses, states = [], 0, 0, {}, []
    for t, ncs in tickets:
        while True:
            res = sg.sg_serve_poll(srv, t, ncs)
            if res is not None:
                break
            time.sleep(0.001)
        lat.append(res["t_done"] - res["t_submit"])
        applies += res["stats"]["applies"]
        ok += res["status"] == sg.SG_OK
        statuses[str(res["status"])] = statuses.get(str(res["status"]), 0) + 1
        states.append(res["psi"])
    wall = time.perf_counter() - t0
    sg.sg_serve_destroy(srv)
    lat = np.array(lat)
    return {"requests": len(reqs), "completed_ok": int(ok), "statuses": statuses,
            "wall_s": wall, "requests_per_s": len(reqs) / wall,
            "instance_applies_per_s": applies / wall,
            "latency_s_p50": float(np.percentile(lat, 50)),
            "latency_s_p99": float(np.percentile(lat, 99))}, states


def serve(sg, window_s, steps_scale, mixed_threshold):
    """The Poisson request stream (20 req/s; D ~ U{3..20}, L ~ U{3..6} capped
    so that N_s <= 5e7; steps ~ U{50..2000}) over its first window_s seconds,
    every request's step count multiplied by steps_scale, in a mixed leg and
    an FP64 leg; each request's mixed result against its FP64 one."""
    import sg_inputs
    reqs = []
    for r in sg_inputs.config4():
        if r.arrival_s >= window_s:
            break
        L = r.inst.L
        while L > 0 and sg.sg_count_sizes(r.inst.D, L)[1] > 5e7:
            L -= 1
        reqs.append({"arrival_s": r.arrival_s, "inst": r.inst, "L": L,
                     "n_cs": sg.sg_count_sizes(r.inst.D, L)[2],
                     "steps": max(1, int(round(r.steps * steps_scale)))})
    # untimed warm-up (first launches of every kernel variant, compile threads)
    serve_leg(sg, [dict(r, steps=1) for r in reqs[:8]], sg.SG_MIXED, mixed_threshold)
    serve_leg(sg, [dict(r, steps=1) for r in reqs[:8]], sg.SG_FP64, -1)
    fp64, s_fp64 = serve_leg(sg, reqs, sg.SG_FP64, -1)
    mixed, s_mixed = serve_leg(sg, reqs, sg.SG_MIXED, mixed_threshold)
    errs = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(s_mixed, s_fp64)]
    return {"workload": "Poisson 20 req/s, D ~ U{3..20}, L ~ U{3..6} (N_s <= 5e7)",
            "window_s": window_s, "steps_scale": steps_scale,
            "mixed_threshold": mixed_threshold,
            "mixed": mixed, "fp64": fp64,
            "request_rel_err_vs_fp64_max": max(errs) if errs else 0.0,
            "request_rel_err_vs_fp64_p50": float(np.percentile(errs, 50)) if errs else 0.0}


def vibronic(sg, steps=100, dt=0.05):
    """The two-state (vibronic) operator of the pyrazine form, 12 modes at
    L = 5: apply throughput, kernel durations, the sweep's roofline figures,
    and a Chebyshev propagation from the displaced Gaussian on the upper
    state with the upper-state population at every 10th step."""
    import torch
    import sg_inputs
    inst = sg_inputs.vibronic_pyrazine(5)
    V = sg.Vibronic.from_instance(inst)
    n = V.n_cs
    x = torch.empty(2 * n, dtype=torch.complex128, device="cuda")
    sg.sg_vibronic_init(V.handle, n, inst.shift, 1, x)
    y = torch.empty_like(x)
    for _ in range(5):
        V.apply(x, y)
    torch.cuda.synchronize()
    reps = 200
    t0 = time.perf_counter()
    for _ in range(reps):
        V.apply(x, y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sg.sg_set_timing(V.problem, True)
    for _ in range(50):
        V.apply(x, y)
    tim = sg.sg_get_timing(V.problem)
    sg.sg_set_timing(V.problem, False)
    sweep_s = tim["sweep_ms"] / max(tim["sweep_launches"], 1) * 1e-3
    reduce_s = tim["reduce_ms"] / max(tim["reduce_launches"], 1) * 1e-3
    flops, nbytes = sg.sg_vibronic_figures(V.handle)
    lo, hi = sg.sg_vibronic_bounds(V.handle, 40)
    psi = x.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, st, pop = sg.sg_vibronic_propagate(V.handle, n, psi, dt, steps, lo, hi, tol=1e-6,
                                               check_every=10)
    torch.cuda.synchronize()
    el_p = time.perf_counter() - t0
    info = V.info
    V.close()
    return {"workload": "two-state pyrazine form, 12 modes, L=5 (N_cs=%d per state, %d terms), FP64"
                        % (n, info["n_terms"]),
            "applies_per_s": reps / el,
            "kernel_avg_us": {"term_sweep": sweep_s * 1e6, "reduce": reduce_s * 1e6},
            "sweep_flops_per_launch": flops, "sweep_bytes_per_launch": nbytes,
            "sweep_flop_frac": flops / sweep_s / 1e12 / FP64_PEAK_TFLOPS,
            "sweep_hbm_frac": nbytes / sweep_s / 1e9 / HBM_PEAK_GBS,
            "propagation": {"steps": steps, "dt": dt, "seconds": el_p, "status": int(status),
                            "applies": st["applies"], "norm_drift": st["max_norm_drift"],
                            "energy_drift": st["max_energy_drift"],
                            "upper_state_population_every_10_steps": [float(v) for v in pop]}}


def tabulated(sg, steps=100, dt=0.05):
    """A general (non-polynomial) coupling potential tabulated on the term
    grids, D = 8, L = 6: host tabulation time, apply throughput, kernel
    durations, the sweep's roofline figures (its bytes include the V_eff
    tables) and a Chebyshev propagation from the displaced Gaussian."""
    import torch
    import sg_inputs
    inst, V = sg_inputs.tabulated_d8_l6()
    P = sg.Problem.from_instance(inst)
    t0 = time.perf_counter()
    sg.sg_set_potential(P.handle, V.at_points)
    t_tab = time.perf_counter() - t0
    info = sg.sg_problem_info(P.handle)
    n = P.n_cs
    x = torch.empty(n, dtype=torch.complex128, device="cuda")
    sg.sg_init_gaussian(P.handle, inst.shift, x)
    y = torch.empty_like(x)
    for _ in range(5):
        P.apply(x, y)
    torch.cuda.synchronize()
    reps = 500
    t0 = time.perf_counter()
    for _ in range(reps):
        P.apply(x, y)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    lo, hi = sg.sg_spectral_bounds(P.handle, 40)
    sweep_s, reduce_s, _ = kernel_times(sg, P, x, dt, 20, lo, hi, sg.SG_FP64, 10)
    el_p, status, st, _ = timed_propagation(sg, P, x, dt, steps, 5, lo, hi, sg.SG_FP64, 10)
    flops, nbytes = info["sweep_flops_fp64"], info["sweep_bytes"]
    P.close()
    return {"workload": "general potential (cosine and Gaussian pair terms) tabulated on the term "
                        "grids, D=8, L=6 (N_cs=%d, %d terms, %d V_eff values), FP64"
                        % (n, info["n_terms"], info["grid_active"]),
            "tabulate_s": t_tab, "potential_evaluations": info["grid_literal"],
            "applies_per_s": reps / el,
            "kernel_avg_us": {"term_sweep": sweep_s * 1e6, "reduce": reduce_s * 1e6},
            "sweep_flops_per_launch": flops, "sweep_bytes_per_launch": nbytes,
            "sweep_flop_frac": flops / sweep_s / 1e12 / FP64_PEAK_TFLOPS,
            "sweep_hbm_frac": nbytes / sweep_s / 1e9 / HBM_PEAK_GBS,
            "propagation": {"steps": steps, "dt": dt, "seconds": el_p, "status": int(status),
                            "applies": st["applies"], "norm_drift": st["max_norm_drift"],
                            "energy_drift": st["max_energy_drift"]}}


def apply_only(sg, args, inst):
    """N applies of the workload's operator (for the profiler), then exit."""
    import torch
    if args.workload == "tab_d8_l6":
        inst, V = inst
        P = sg.Problem.from_instance(inst)
        sg.sg_set_potential(P.handle, V.at_points)
        x = torch.empty(P.n_cs, dtype=torch.complex128, device="cuda")
        sg.sg_init_gaussian(P.handle, inst.shift, x)
        y = torch.empty_like(x)
        for _ in range(args.apply_only):
            P.apply(x, y)
        torch.cuda.synchronize()
        P.close()
        print(json.dumps({"apply_only": args.apply_only, "workload": args.workload}), flush=True)
        return
    if args.workload == "vib_d12_l5":
        V = sg.Vibronic.from_instance(inst)
        x = torch.empty(2 * V.n_cs, dtype=torch.complex128, device="cuda")
        sg.sg_vibronic_init(V.handle, V.n_cs, inst.shift, 1, x)
        y = torch.empty_like(x)
        for _ in range(args.apply_only):
            V.apply(x, y)
        torch.cuda.synchronize()
        V.close()
        print(json.dumps({"apply_only": args.apply_only, "workload": args.workload}), flush=True)
        return
    P = sg.Problem.from_instance(inst)
    psi = torch.empty(P.n_cs, dtype=torch.complex128, device="cuda")
    sg.sg_init_gaussian(P.handle, inst.shift, psi)
    y = torch.empty_like(psi)
    prec = sg.SG_FP64 if (args.precision or "fp64") == "fp64" else sg.SG_MIXED
    for _ in range(args.apply_only):
        P.apply(psi, y, prec)
    torch.cuda.synchronize()
    P.close()
    print(json.dumps({"apply_only": args.apply_only, "workload": args.workload,
                      "precision": "fp64" if prec == sg.SG_FP64 else "mixed"}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="Chebyshev steps timed (default: the workload's, 500 at D=12 L=6)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d12_l6", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"],
                    help="default: mixed (tuned) for d12_l6, fp64 otherwise")
    ap.add_argument("--latency-samples", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the (6,6), propagator, batched and serving sections")
    ap.add_argument("--no-error-curve", action="store_true")
    ap.add_argument("--forced-curve-steps", type=int, default=100)
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-latency-steps", type=int, default=20)
    ap.add_argument("--serve-window", type=float, default=3.0)
    ap.add_argument("--serve-steps-scale", type=float, default=0.2)
    ap.add_argument("--serve-mixed-threshold", type=int, default=0)
    ap.add_argument("--grid-kinetic", action="store_true",
                    help="SG_FP64 in the literal form (kinetic matrices on every term grid) "
                         "instead of the default exact diagonal split")
    ap.add_argument("--apply-only", type=int, default=0, metavar="N",
                    help="only build the workload and run N applies (for the profiler)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (the "
                         "reference kernel for scaling HBM byte counters) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; term sharding across GPUs "
                                   "is not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": nbytes, "bytes_written": nbytes,
                          "launches": 3}), flush=True)
        return
    import paper_2111_13655_amd as sg

    wl = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = wl["steps"]
    if args.precision is None:
        args.precision = "mixed" if args.workload == "d12_l6" else "fp64"
    inst = instance_for(args.workload)
    torch.cuda.set_device(torch.device("cuda", 0))
    if args.apply_only > 0:
        apply_only(sg, args, inst)
        return
    if args.workload in ("vib_d12_l5", "tab_d8_l6"):
        sys.exit("this workload is profiled with --apply-only; its bench figures are a "
                 "section of the default run")
    out = headline(sg, args, wl, inst)
    if not args.no_extras:
        if args.workload != "d6_l6":
            log("[bench] D=6 L=6 FP64 trajectory")
            out["d6_l6_fp64"] = d6l6_leg(sg)
            log(f"[bench] {out['d6_l6_fp64']}")
        log("[bench] two-state (vibronic) pyrazine form, 12 modes, L=5")
        out["vibronic"] = vibronic(sg)
        log(f"[bench] {out['vibronic']}")
        log("[bench] tabulated general potential, D=8 L=6")
        out["tabulated"] = tabulated(sg)
        log(f"[bench] {out['tabulated']}")
        log("[bench] propagators (D=6, L=6)")
        out["propagators"] = propagators(sg)
        log(f"[bench] {out['propagators']}")
        log(f"[bench] batched (64 instances, {args.batch_steps} steps, mixed and fp64)")
        out["batched"] = batched(sg, args.batch_steps, args.batch_latency_steps)
        log(f"[bench] { {k: v for k, v in out['batched'].items() if k != 'final_state_rel_err_vs_fp64'} }")
        log("[bench] serving (mixed and fp64 legs)")
        out["serve"] = serve(sg, args.serve_window, args.serve_steps_scale,
                             args.serve_mixed_threshold)
        log(f"[bench] {out['serve']}")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
        log(f"[bench] {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
