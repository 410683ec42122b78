"""Benchmark: one full pressure solve of the 256x256x512 bubbly duct per step.

A step is the whole path on resident inputs: mixture density from the gas
fraction, right-hand side from the face velocities, face coefficients and the
multigrid hierarchy (pp_set_density), and the solve to a relative residual of
1e-10 from a zero initial guess (pp_solve).  The headline form is float64
flexible CG preconditioned by a float32 multigrid cycle (float32-refined); the
plain float64 form is timed the same way for the speed-up.

Prints one JSON line (rank 0).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-10 residual & cells·iters/s (HBM GB/s %peak); FP32-refined vs FP64; p50/p99"
HBM_PEAK_GBS = 8000.0
HERE = os.path.dirname(os.path.abspath(__file__))


def csrc_sha256():
    """Hash of the kernel and launch sources (the HBM-traffic profile is valid for these only)."""
    h = hashlib.sha256()
    d = os.path.join(HERE, "paper_2104_01636_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(d, "*.hpp")) + glob.glob(os.path.join(d, "*.hip"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter profile of `workload`, or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(HERE, "profiles", f"hbm_traffic_{workload}.md")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        m = re.search(r"kernel: (\S+)\s+traffic_bytes_per_launch: (\d+)\s+source_sha256: ([0-9a-f]+)", fh.read())
    if not m or m.group(1) != kernel or m.group(3) != csrc_sha256():
        return None
    return int(m.group(2))


def pct(a, q):
    return float(np.percentile(np.asarray(a), q))


def serving_leg(args, dev, log):
    """Serving workload: independent duct cases of mixed sizes arriving as a Poisson
    stream, solved (refined form, 1e-8) by the library's request loop."""
    import ctypes

    import torch
    from paper_2104_01636_amd import ppsolve, serve, workload as W

    t0 = time.time()
    reqs = W.serving_requests(args.serving_requests, rate_hz=args.serving_rate, seed=4)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    items, keep = [], []
    for r in reqs:
        nx, ny, nz = r["grid"]
        c = W.make_case(nx, ny, nz, r["n_bubbles"], r["diameter"], seed=r["seed"])
        rho_t = ppsolve.density_from_fraction(g(c.alpha))
        rhs_t = ppsolve.divergence(g(c.u), g(c.v), g(c.w), c.h)
        out_t = torch.empty_like(rhs_t)
        keep.append((rho_t, rhs_t, out_t))
        items.append(dict(arrival_s=r["arrival_s"], case_id=r["index"],
                          cfg=ppsolve.make_config(nx, ny, nz, c.h, "fp32_refined", 1e-8, 4000),
                          rho=ctypes.c_void_p(rho_t.data_ptr()), rhs=ctypes.c_void_p(rhs_t.data_ptr()),
                          p_out=ctypes.c_void_p(out_t.data_ptr())))
    torch.cuda.synchronize()
    log(f"serving: {len(items)} requests generated in {time.time() - t0:.1f}s")
    with serve.Server(int(args.serving_budget_gb * (1 << 30)), slots=args.serving_slots) as srv:
        res = serve.replay(srv, items)
        st = srv.stats()
    bad = [r for r in res if r["status"] != 0]
    iters = [r["stats"]["inner_iters_total"] for r in res if r["status"] == 0]
    out = {"requests": len(items), "rate_per_s": args.serving_rate, "slots": args.serving_slots,
           "budget_gb": args.serving_budget_gb, "tol": 1e-8, "form": "fp32_refined",
           "latency_p50_ms": round(st["latency_p50_ms"], 3), "latency_p99_ms": round(st["latency_p99_ms"], 3),
           "latency_max_ms": round(st["latency_max_ms"], 3), "solves_per_s": round(st["solves_per_s"], 2),
           "max_concurrent": st["max_running"], "evictions": st["evictions"],
           "peak_resident_gb": round(st["peak_resident_bytes"] / (1 << 30), 3), "failed": len(bad),
           "inner_iters_median": int(np.median(iters)) if iters else None}
    log(f"serving: {out}")
    return out


def next_rows_leg(args, case, log, alpha_t, u_t, v_t, w_t, rho_t, rhs_t, p_t):
    """The steps on either side of the solve and the paper's own solver form, on the same input.

    * Time per call of the mixture density, the divergence (step 11's right-hand side), the face
      projection (step 12) and the surface-tension right-hand side (eq. ppe_surface_tension):
      torch events on the current stream, which is the stream the library launches them on,
      around repeated calls.  Each call ends by synchronising its stream, so the time per call
      includes one launch gap; the rates are algorithmic bytes (each array element read or
      written once) over that time, a lower bound on the kernel's own rate.
    * Multigrid as the solver (red-black SOR V-cycles, no CG; Section 2.1) in float64, to the
      same tolerance from a zero guess, for SOR factors 1.0 and 1.15."""
    import torch
    from paper_2104_01636_amd import ppsolve

    n = case.n_cells
    reps = 10
    kappa_t = torch.full_like(alpha_t, 2.0 / (0.5 * case.diameter * case.h))  # curvature of a bubble
    out_t = torch.empty_like(alpha_t)
    u2, v2, w2 = u_t.clone(), v_t.clone(), w_t.clone()
    calls = {  # name: (launch, algorithmic bytes per cell)
        "density_from_fraction": (lambda: ppsolve.density_from_fraction(alpha_t, 1000.0, 1.2, out=out_t), 16),
        "divergence": (lambda: ppsolve.divergence(u_t, v_t, w_t, case.h, 1.0, out=out_t), 32),
        "project": (lambda: ppsolve.project(rho_t, p_t, u2, v2, w2, case.h, 1e-3), 64),
        "surface_tension_rhs": (lambda: ppsolve.surface_tension_rhs(rho_t, alpha_t, kappa_t, 0.072, case.h,
                                                                    out=out_t), 32),
    }
    kern = {}
    for name, (call, bpc) in calls.items():
        call()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = bpc * n / (us * 1e-6) / 1e9
        kern[name] = {"us_per_call": round(us, 2), "calls": reps, "bytes_per_cell": bpc, "GB_per_s": round(gbs, 1),
                      "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"next rows: {name} {us:.1f} us, {gbs:.0f} GB/s")
    del u2, v2, w2, kappa_t, out_t

    mg = {}
    for omega in (1.0, 1.15):
        with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=args.tol, max_iters=4000,
                            flags=ppsolve.PP_FLAG_MG_SOLVER, omega=omega) as S:
            S.set_density(rho_t)
            times = []
            for k in range(2):  # the first solve is a warm-up
                p_t.zero_()
                torch.cuda.synchronize()
                a = time.perf_counter()
                _, st = S.solve(rhs_t, p_t)
                torch.cuda.synchronize()
                if k:
                    times.append((time.perf_counter() - a) * 1e3)
            mg[f"omega_{omega:g}"] = {"time_to_tol_ms": round(times[0], 3), "cycles": int(st["iters"]),
                                      "ms_per_cycle": round(st["solve_ms"] / max(1, st["iters"]), 4),
                                      "rel_residual": float(f"{st['rel_residual']:.3e}")}
            log(f"next rows: multigrid solver omega {omega:g}: {times[0]:.1f} ms, {st['iters']} cycles, "
                f"residual {st['rel_residual']:.2e}")
    return {"around_the_solve": kern, "multigrid_solver_fp64": mg}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="duct256")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=120, help="oracle iterations in the CPU-baseline sample")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for hardware traffic counters)")
    ap.add_argument("--forms", default="fp32_refined,fp64")
    ap.add_argument("--kernel-timing", choices=("timed", "separate"), default="timed",
                    help="timed: HIP events around every finest-level kernel during the timed steps (launched "
                         "directly); separate: timed steps replay HIP graphs, events in extra profiling steps")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving leg (Poisson arrivals, mixed grids); 0 skips it")
    ap.add_argument("--serving-rate", type=float, default=40.0)
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the kernels around the solve and the multigrid-as-solver form")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-budget-gb", type=float, default=24.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the solver runs on one GPU (the solve is not sharded across GPUs); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_01636_amd import ppsolve, workload as W

    def log(*a):
        print("[bench]", *a, file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    case = W.preset(args.workload)
    n = case.n_cells
    log(f"workload {args.workload}: {case.nx}x{case.ny}x{case.nz}, {len(case.centres)} bubbles d={case.diameter}, "
        f"void {case.alpha.mean():.4f}, generated in {time.time() - t0:.1f}s")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    alpha_t, u_t, v_t, w_t = g(case.alpha), g(case.u), g(case.v), g(case.w)
    rho_t = torch.empty_like(alpha_t)
    rhs_t = torch.empty_like(alpha_t)
    p_t = torch.zeros_like(alpha_t)
    torch.cuda.synchronize()

    def step(S):
        ppsolve.density_from_fraction(alpha_t, 1000.0, 1.2, out=rho_t)
        ppsolve.divergence(u_t, v_t, w_t, case.h, 1.0, out=rhs_t)
        S.set_density(rho_t)
        p_t.zero_()
        _, st = S.solve(rhs_t, p_t)
        return st

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 2 x 1 GiB device-to-device copies (read 1 GiB + write 1 GiB each)")
        del src, dst

    results = {}
    forms = args.forms.split(",")
    for mode in forms:
        S = ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=args.tol, max_iters=4000)
        for _ in range(args.warmup):
            step(S)
        torch.cuda.synchronize()
        times, stats = [], []
        if args.kernel_timing == "timed":
            S.timing(1)
        T0 = time.perf_counter()
        for k in range(args.steps):
            a = time.perf_counter()
            st = step(S)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - a) * 1e3)
            stats.append(st)
        torch.cuda.synchronize()
        T1 = time.perf_counter()
        if args.kernel_timing == "separate":
            S.timing(1)
            for _ in range(2):
                step(S)
            torch.cuda.synchronize()
        kt = S.timing(0)
        S.timing(-1)
        iters = [st["inner_iters_total"] if mode == "fp32_refined" else st["iters"] for st in stats]
        results[mode] = dict(total_s=T1 - T0, times=times, stats=stats, iters=iters, kernels=kt,
                             p=p_t.detach().cpu().numpy().copy())
        log(f"{mode}: step ms p50 {pct(times, 50):.2f} p99 {pct(times, 99):.2f}; iters {iters[0]} "
            f"(outer {stats[0]['outer_iters']}); residual {stats[0]['rel_residual']:.2e}; "
            f"setup {stats[0]['setup_ms']:.2f} ms; solve {stats[0]['solve_ms']:.2f} ms")
        S.close()

    head = results[forms[0]]
    ms_per_step = head["total_s"] * 1e3 / args.steps
    iters = int(np.median(head["iters"]))
    value = n * sum(head["iters"]) / head["total_s"]

    # agreement of the two forms (both zero-mean)
    diff_modes = None
    if "fp32_refined" in results and "fp64" in results:
        pa, pb = results["fp32_refined"]["p"], results["fp64"]["p"]
        diff_modes = float(np.max(np.abs(pa - pb)) / np.max(np.abs(pb)))
        log(f"refined vs fp64 L-inf {diff_modes:.2e}")

    # roofline of the dominant kernel (largest total device time among the timed finest-level kernels)
    kt = head["kernels"] or {}
    roof = None
    if kt:
        name, (ms, launches, bytes_) = max(kt.items(), key=lambda kv: kv[1][0])
        avg_ms = ms / launches
        achieved = bytes_ / launches / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "timing": ("HIP events on the solver's stream around each launch, during the timed steps"
                           if args.kernel_timing == "timed" else
                           "HIP events on the solver's stream around each launch, 2 extra steps after the timed ones"),
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(name, args.workload),
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
                "avg_launch_us": round(avg_ms * 1e3, 2), "launches": int(launches),
                "algorithmic_bytes_per_launch": int(bytes_ / launches)}
        kern_tab = {k: {"avg_us": round(v[0] / v[1] * 1e3, 2), "launches": int(v[1]),
                        "GB_per_s": round(v[2] / v[1] / (v[0] / v[1] * 1e-3) / 1e9, 1),
                        "share_of_step": round(v[0] / (head["total_s"] * 1e3), 3)} for k, v in kt.items()}
    else:
        kern_tab = {}

    next_rows = None
    if not args.no_next_rows:
        next_rows = next_rows_leg(args, case, log, alpha_t, u_t, v_t, w_t, rho_t, rhs_t, p_t)

    serving = None
    if args.serving_requests > 0:
        serving = serving_leg(args, dev, log)

    cpu = None
    if not args.no_cpu_baseline:
        # CPU baseline: the float64 oracle on the same input, a bounded number of iterations
        from oracle import cref, poisson as P
        rho = P.density_from_fraction(case.alpha)
        b = P.divergence(case.u, case.v, case.w, case.h)
        nthreads = cref.num_threads()
        t = time.perf_counter()
        _, it, _, secs = cref.solve(rho, b, case.h, tol=1e-30, maxit=args.cpu_iters)
        cpu = {"value": round(n * it / secs, 1), "unit": "cells*iters/s", "cores": nthreads, "kind": "oracle",
               "sample": f"{it} MG-preconditioned CG iterations of the float64 C/OpenMP oracle on the full "
                         f"{case.nx}x{case.ny}x{case.nz} input ({secs:.1f} s incl. its hierarchy set-up)",
               "host_cpu": platform.processor() or platform.machine()}
        log(f"cpu baseline: {cpu['value']:.3e} cells*iters/s on {nthreads} threads ({time.perf_counter() - t:.1f}s)")

    tt = {m: results[m]["times"] for m in results}
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cells*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"bubbly duct {case.nx}x{case.ny}x{case.nz}, {len(case.centres)} bubbles "
                               f"d={case.diameter:g} cells, rho 1000/1.2, solve to rel. residual {args.tol:g}",
                   "cells": n, "bubbles": len(case.centres), "form": forms[0], "seed": case.seed},
        "time_to_tol_ms": {m: {"p50": round(pct(t, 50), 3), "p99": round(pct(t, 99), 3)} for m, t in tt.items()},
        "speedup_fp32_refined_vs_fp64": (round(pct(tt["fp64"], 50) / pct(tt["fp32_refined"], 50), 3)
                                         if "fp64" in tt and "fp32_refined" in tt else None),
        "iters": {m: {"krylov": int(np.median(results[m]["iters"])),
                      "outer": int(results[m]["stats"][0]["outer_iters"])} for m in results},
        "setup_ms": round(head["stats"][0]["setup_ms"], 3),
        "rel_residual": {m: float(f"{results[m]['stats'][-1]['rel_residual']:.3e}") for m in results},
        "linf_refined_vs_fp64": float(f"{diff_modes:.3e}") if diff_modes is not None else None,
        "cells_per_s_solved": round(n / (ms_per_step * 1e-3), 1),
        "roofline": roof,
        "kernels": kern_tab,
        "next_rows": next_rows,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
