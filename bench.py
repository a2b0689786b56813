"""Benchmark of the Smolyak H|psi> hot path on one MI355X.

Default workload: the (D, L) = (6, 6) coupled-anharmonic Hamiltonian
(omega ~ U(0.5, 2), c ~ U(-0.05, 0.05), k ~ U(-0.02, 0.02), seeded), a
displaced-Gaussian wave packet propagated by Chebyshev steps of dt = 0.05 in
FP64, with norm and energy checked every 100 steps.  One benchmark "step" is
one Chebyshev time step: K-1 applications of H_S (term sweep + fixed-order
reduce with the recurrence fused into it) over the whole term set.

Prints ONE JSON line: applies/s (value), grid-points/s (literal and active
counts), p50/p99 latency of a single apply, the dominant kernel's roofline
(term sweep, FP64 VALU), and the CPU oracle's rate on a bounded sample.
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

FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# Sources whose change invalidates recorded HBM counters of the sweep kernel.
KERNEL_SOURCES = ["paper_2111_13655_amd/csrc/sg_sweep.hip", "paper_2111_13655_amd/csrc/sg_internal.h",
                  "paper_2111_13655_amd/csrc/sg_plan.cpp", "paper_2111_13655_amd/csrc/sg_terms.cpp"]

WORKLOADS = {
    "d6_l6_fp64": dict(D=6, L=6, dt=0.05, check_every=100, precision="fp64",
                       desc="smolyak H|psi> D=6 L=6 coupled anharmonic, Chebyshev dt=0.05, FP64"),
    "d2_l4_fp64": dict(D=2, L=4, dt=0.1, check_every=10, precision="fp64",
                       desc="smolyak H|psi> D=2 L=4 coupled anharmonic, Chebyshev dt=0.1, FP64"),
    "d12_l6_mixed": dict(D=12, L=6, dt=0.05, check_every=1, precision="mixed",
                         desc="smolyak H|psi> D=12 L=6 coupled anharmonic, Chebyshev dt=0.05, mixed"),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def instance_for(name):
    import sg_inputs
    return {"d6_l6_fp64": sg_inputs.config1, "d2_l4_fp64": sg_inputs.config0,
            "d12_l6_mixed": sg_inputs.config2}[name]()


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


def cpu_baseline(inst, info, budget_s: float):
    """The FP64 oracle's literal Alg. 1 (test infrastructure) on a bounded
    sample: as many whole applies as fit in about budget_s seconds."""
    from oracle.action import Oracle
    try:
        from threadpoolctl import threadpool_info
        blas_threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        blas_threads = 1
    O = Oracle(inst)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(O.S.n_cs) + 1j * rng.standard_normal(O.S.n_cs)
    n = 0
    t0 = time.perf_counter()
    while True:
        psi = O.apply_literal(psi)
        psi /= np.linalg.norm(psi)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    rate = n / dt
    return {"value": rate, "unit": "applies/s", "cores": int(blas_threads),
            "kind": "oracle",
            "sample": f"{n} whole FP64 applies of the literal per-term oracle (Alg. 1) on the "
                      f"same operator, {dt:.1f} s; host affinity {len(os.sched_getaffinity(0))} cpus",
            "grid_pts_per_s_literal": rate * info["grid_literal"]}


def _throughput(sg, P, prec, reps):
    """Back-to-back applies between two events on the current stream: applies/s."""
    import torch
    n = P.n_cs
    x = torch.zeros(n, dtype=torch.complex128, device="cuda")
    x[0] = 1.0
    y = torch.empty_like(x)
    for _ in range(3):
        P.apply(x, y, prec)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        P.apply(x, y, prec)
    e1.record()
    e1.synchronize()
    return reps / (e0.elapsed_time(e1) * 1e-3)


def mixed_vs_fp64(sg, reps=20, prop_steps=20):
    """(D, L) = (12, 6): the precision autotuner's choice at the 1e-6 bar, its
    measured error against the FP64 apply, both throughputs, and the error of
    a mixed-precision propagation against the FP64 one after every step."""
    import torch
    import sg_inputs
    inst = sg_inputs.config2()
    P = sg.Problem.from_instance(inst)
    n = P.n_cs
    psi = torch.empty(n, dtype=torch.complex128, device="cuda")
    sg.sg_init_gaussian(P.handle, inst.shift, psi)
    thr, err_tuned = sg.sg_tune_mixed(P.handle, psi, 1e-6, 3)
    # error on an independent random state
    rng = np.random.default_rng(7)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x = torch.from_numpy(v / np.linalg.norm(v)).to("cuda")
    y64, y32 = torch.empty_like(x), torch.empty_like(x)
    P.apply(x, y64, sg.SG_FP64)
    P.apply(x, y32, sg.SG_MIXED)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64))
    t64 = _throughput(sg, P, sg.SG_FP64, reps)
    t32 = _throughput(sg, P, sg.SG_MIXED, reps)
    # propagation from the displaced Gaussian in both precisions, step by
    # step: relative distance of the mixed state from the FP64 one
    lo, hi = sg.sg_spectral_bounds(P.handle, 40)

    def prop_errors():
        a64, a32 = psi.clone(), psi.clone()
        errs = []
        for _ in range(prop_steps):
            sg.sg_propagate_chebyshev(P.handle, a64, 0.05, 1, lo, hi, tol=0.0)
            sg.sg_propagate_chebyshev(P.handle, a32, 0.05, 1, lo, hi, tol=0.0,
                                      precision=sg.SG_MIXED)
            errs.append(float(torch.linalg.norm(a32 - a64) / torch.linalg.norm(a64)))
        return errs

    step_err = prop_errors()
    # the same with every |D_l| = 1 term in FP32 (the tuner's bar aside)
    sg.sg_set_mixed_threshold(P.handle, 1)
    step_err_1 = prop_errors()
    sg.sg_set_mixed_threshold(P.handle, thr)
    info = sg.sg_problem_info(P.handle)
    P.close()
    return {"workload": "D=12 L=6 coupled anharmonic (same family), one apply",
            "fp64_applies_per_s": t64, "mixed_applies_per_s": t32, "speedup": t32 / t64,
            "mixed_threshold": thr, "rel_err_vs_fp64_tuning_state": err_tuned,
            "rel_err_vs_fp64_random_state": err, "tol": 1e-6,
            "propagation_dt": 0.05, "propagation_rel_err_per_step": step_err,
            "propagation_max_rel_err": max(step_err) if step_err else 0.0,
            "propagation_rel_err_per_step_threshold_1": step_err_1,
            "grid_pts_per_s_active_mixed": t32 * info["grid_active"]}


def propagators(sg, steps=40, dt=0.05):
    """(D, L) = (6, 6), FP64: the Taylor, Runge-Kutta, short-iterative-Lanczos
    and Bulirsch-Stoer propagators against Chebyshev over the same span, from the
    displaced Gaussian: wall time, applies, and the distance of each final
    state from the Chebyshev one (converged to 1e-16 per step)."""
    import time
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
                     "rel_diff_vs_chebyshev": float(torch.linalg.norm(x - ref) /
                                                    torch.linalg.norm(ref))}
    P.close()
    return out


def batched(sg, steps):
    """64 independent instances (D ~ U{4..10}, L ~ U{4..7}) advanced together
    in mixed precision: instance-applies/s over a bounded number of steps."""
    import torch
    import sg_inputs
    insts = sg_inputs.config3()
    probs = [sg.Problem.from_instance(i) for i in insts]
    psis, lo, hi = [], [], []
    for P, inst in zip(probs, insts):
        x = torch.empty(P.n_cs, dtype=torch.complex128, device="cuda")
        sg.sg_init_gaussian(P.handle, inst.shift, x)
        psis.append(x)
        a, b = sg.sg_spectral_bounds(P.handle, 40)
        lo.append(a)
        hi.append(b)
    b = sg.sg_batch_create([P.handle for P in probs])
    dts = [i.meta["dt"] for i in insts]
    sg.sg_batch_propagate(b, psis, dts, 1, lo, hi, tol=1e-6, precision=sg.SG_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, st = sg.sg_batch_propagate(b, psis, dts, steps, lo, hi, tol=1e-6,
                                       precision=sg.SG_MIXED, check_every=steps,
                                       use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    applies = sum(s["applies"] for s in st)
    grid = sum(P.info["grid_active"] * s["applies"] for P, s in zip(probs, st))
    sg.sg_batch_free(b)
    for P in probs:
        P.close()
    return {"workload": "64 instances, D ~ U{4..10}, L ~ U{4..7}, mixed, dt = 0.05",
            "steps": steps, "status": int(status), "seconds": dt,
            "instance_applies_per_s": applies / dt, "grid_pts_per_s_active": grid / dt,
            "ms_per_batched_step": dt / steps * 1e3}


def serve(sg, window_s, steps_scale):
    """The Poisson request stream (20 req/s; D ~ U{3..20}, L ~ U{3..6} capped
    so that N_s <= 5e7; steps ~ U{50..2000}) over its first window_s seconds,
    every request's step count multiplied by steps_scale so that the sample
    drains in bounded time.  Requests are submitted at their arrival times
    and stay resident until done; latency is submit -> result."""
    import sg_inputs
    reqs = [r for r in sg_inputs.config4() if r.arrival_s < window_s]
    # FP32 only for the |D_l| = 1 terms: the server applies one precision
    # policy to every request, and larger thresholds exceed the 1e-6 drift
    # gate at the largest D of the stream
    srv = sg.sg_serve_create(max_slots=64, precision=sg.SG_MIXED, check_every=100, tol=1e-6,
                             mixed_threshold=1, compile_threads=8)
    tickets = []
    t0 = time.perf_counter()
    for r in reqs:
        inst = r.inst
        L = inst.L
        while L > 0 and sg.sg_count_sizes(inst.D, L)[1] > 5e7:
            L -= 1
        now = time.perf_counter() - t0
        if r.arrival_s > now:
            time.sleep(r.arrival_s - now)
        nsteps = max(1, int(round(r.steps * steps_scale)))
        tickets.append((sg.sg_serve_submit(srv, inst.D, L, inst.omega, inst.c, inst.k,
                                           inst.shift, 0.05, nsteps), nsteps))
    lat, applies, ok, statuses = [], 0, 0, {}
    for t, _ in tickets:
        while True:
            res = sg.sg_serve_poll(srv, t)
            if res is not None:
                break
            time.sleep(0.001)
        lat.append(res["t_done"] - res["t_submit"])
        applies += res["stats"]["applies"]
        ok += res["status"] == sg.SG_OK
        statuses[str(res["status"])] = statuses.get(str(res["status"]), 0) + 1
    wall = time.perf_counter() - t0
    sg.sg_serve_destroy(srv)
    lat = np.array(lat)
    return {"workload": "Poisson 20 req/s, D ~ U{3..20}, L ~ U{3..6} (N_s <= 5e7), mixed",
            "window_s": window_s, "steps_scale": steps_scale, "requests": len(reqs),
            "completed_ok": int(ok), "statuses": statuses, "wall_s": wall, "requests_per_s": len(reqs) / wall,
            "instance_applies_per_s": applies / wall,
            "latency_s_p50": float(np.percentile(lat, 50)),
            "latency_s_p99": float(np.percentile(lat, 99))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="d6_l6_fp64", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed"])
    ap.add_argument("--latency-samples", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the mixed-vs-FP64, batched and serving sections")
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--serve-window", type=float, default=3.0)
    ap.add_argument("--serve-steps-scale", type=float, default=0.05)
    ap.add_argument("--grid-kinetic", action="store_true",
                    help="SG_FP64 in the literal form (kinetic matrices on every term grid) "
                         "instead of the default exact diagonal split")
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
    prec_name = args.precision or wl["precision"]
    prec = sg.SG_FP64 if prec_name == "fp64" else sg.SG_MIXED
    inst = instance_for(args.workload)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    log(f"[bench] build {args.workload} D={inst.D} L={inst.L}")
    P = sg.Problem.from_instance(inst)
    if args.grid_kinetic:
        sg.sg_set_operator_form(P.handle, True)
    info = sg.sg_problem_info(P.handle)
    n = P.n_cs
    psi0 = torch.empty(n, dtype=torch.complex128, device=dev)
    sg.sg_init_gaussian(P.handle, inst.shift, psi0)
    emin, emax = sg.sg_spectral_bounds(P.handle, 40)
    log(f"[bench] N_cs={n} N_st={info['n_terms']} N_s={info['n_s']} bounds=({emin:.3f},{emax:.3f})")

    # warmup
    psi = psi0.clone()
    if args.warmup > 0:
        sg.sg_propagate_chebyshev(P.handle, psi, wl["dt"], args.warmup, emin, emax, tol=1e-6,
                                  precision=prec, check_every=wl["check_every"])
    torch.cuda.synchronize()

    # timed region: K Chebyshev steps
    psi = psi0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    status, stats, ntr, etr = sg.sg_propagate_chebyshev(
        P.handle, psi, wl["dt"], args.steps, emin, emax, tol=1e-6, precision=prec,
        check_every=wl["check_every"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    applies = stats["applies"]
    log(f"[bench] timed {args.steps} steps: {elapsed:.3f} s, {applies} applies, status {status}")

    # kernel durations over the same K steps (events around every launch)
    psi_t = psi0.clone()
    sg.sg_set_timing(P.handle, True)
    sg.sg_propagate_chebyshev(P.handle, psi_t, wl["dt"], args.steps, emin, emax, tol=1e-6,
                              precision=prec, check_every=wl["check_every"])
    tim = sg.sg_get_timing(P.handle)
    sg.sg_set_timing(P.handle, False)
    sweep_avg_s = tim["sweep_ms"] / max(tim["sweep_launches"], 1) * 1e-3
    reduce_avg_s = tim["reduce_ms"] / max(tim["reduce_launches"], 1) * 1e-3
    info = sg.sg_problem_info(P.handle)
    sweep_flops = info["sweep_flops_fp64"] if prec == sg.SG_FP64 else info["sweep_flops_mixed"]
    achieved_tflops = sweep_flops / sweep_avg_s / 1e12
    peak = FP64_VALU_PEAK_TFLOPS
    log(f"[bench] sweep avg {sweep_avg_s * 1e6:.2f} us, reduce avg {reduce_avg_s * 1e6:.2f} us")

    # per-apply latency
    x = psi0.clone()
    y = torch.empty_like(x)
    lat = []
    for _ in range(min(50, args.latency_samples)):
        P.apply(x, y, prec)
    torch.cuda.synchronize()
    for _ in range(args.latency_samples):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        P.apply(x, y, prec)
        e1.record()
        e1.synchronize()
        lat.append(e0.elapsed_time(e1) * 1e3)
    lat = np.array(lat)

    value = applies / elapsed
    out = {
        "metric": "H|psi> applies/s and grid-pts/s vs plain FP64 at 1e-6 rel err; p50/p99 latency",
        "value": value,
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / max(args.steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64" if prec == sg.SG_FP64 else "f32+f64",
        "data": "synthetic (seeded coupled-anharmonic Hamiltonian, displaced Gaussian)",
        "config": {"workload": wl["desc"], "D": inst.D, "L": inst.L, "dt": wl["dt"],
                   "precision": prec_name, "n_terms": info["n_terms"], "n_cs": n,
                   "n_s": info["n_s"], "chebyshev_terms": stats["cheb_terms"],
                   "check_every": wl["check_every"], "parallelism": "single GPU",
                   "operator_form": ("split" if (prec == sg.SG_MIXED or info["fp64_split"])
                                     else "grid_kinetic")},
        "grid_pts_per_s_literal": value * info["grid_literal"],
        "grid_pts_per_s_active": value * info["grid_active"],
        "latency_us_p50": float(np.percentile(lat, 50)),
        "latency_us_p99": float(np.percentile(lat, 99)),
        "norm_drift": stats["max_norm_drift"],
        "energy_drift": stats["max_energy_drift"],
        "status": int(status),
        "kernel_avg_us": {"term_sweep": sweep_avg_s * 1e6, "reduce": reduce_avg_s * 1e6},
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved_tflops / peak,
                     "traffic": recorded_traffic(f"{args.workload}/{prec_name}",
                                                 "sweep_kernel<double>"),
                     "kernel": "sweep_kernel",
                     "flops_per_launch": sweep_flops},
    }
    P.close()
    if not args.no_extras:
        log("[bench] mixed vs fp64 (D=12, L=6)")
        out["mixed_vs_fp64"] = mixed_vs_fp64(sg)
        log(f"[bench] {out['mixed_vs_fp64']}")
        log("[bench] propagators (D=6, L=6)")
        out["propagators"] = propagators(sg)
        log(f"[bench] {out['propagators']}")
        log("[bench] batched (64 instances)")
        out["batched"] = batched(sg, args.batch_steps)
        log(f"[bench] {out['batched']}")
        log("[bench] serving")
        out["serve"] = serve(sg, args.serve_window, args.serve_steps_scale)
        log(f"[bench] {out['serve']}")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline")
        out["cpu_baseline"] = cpu_baseline(inst, info, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
