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


def _serving_stats(st, res, extra=None):
    bad = [r for r in res if r["status"] != 0]
    iters = [r["stats"]["inner_iters_total"] for r in res if r["status"] == 0]
    out = {"latency_p50_ms": round(st["latency_p50_ms"], 3), "latency_p99_ms": round(st["latency_p99_ms"], 3),
           "latency_max_ms": round(st["latency_max_ms"], 3), "solves_per_s": round(st["solves_per_s"], 2),
           "max_concurrent": st["max_running"], "evictions": st["evictions"],
           "peak_resident_gb": round(st["peak_resident_bytes"] / (1 << 30), 3), "failed": len(bad),
           "inner_iters_median": int(np.median(iters)) if iters else None}
    out.update(extra or {})
    return out


def serving_leg(args, dev, log):
    """Serving workload: independent duct cases of mixed sizes, solved (refined form, 1e-8) by the
    library's request loop.  Three legs on the same request mix:
      * poisson: the configured stream, Poisson arrivals at 40/s, every request a new case;
      * burst: the same 256 requests all at t = 0 on a fresh server, so solves/s is the capacity;
      * repeat: 32 cases, 8 requests each at the same arrival rate, the later ones without a
        density (the resident hierarchy is reused) and with a perturbed right-hand side (the
        resident pressure is the warm start)."""
    import ctypes

    import torch
    from paper_2104_01636_amd import ppsolve, serve, workload as W

    t0 = time.time()
    reqs = W.serving_requests(args.serving_requests, rate_hz=args.serving_rate, seed=4)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    vp = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None  # noqa: E731
    items, keep, cases = [], [], []
    for r in reqs:
        nx, ny, nz = r["grid"]
        c = W.make_case(nx, ny, nz, r["n_bubbles"], r["diameter"], seed=r["seed"])
        rho_t = ppsolve.density_from_fraction(g(c.alpha))
        rhs_t = ppsolve.divergence(g(c.u), g(c.v), g(c.w), c.h)
        out_t = torch.empty_like(rhs_t)
        keep.append((rho_t, rhs_t, out_t))
        cases.append(c)
        items.append(dict(arrival_s=r["arrival_s"], case_id=r["index"],
                          cfg=ppsolve.make_config(nx, ny, nz, c.h, "fp32_refined", 1e-8, 4000),
                          rho=vp(rho_t), rhs=vp(rhs_t), p_out=vp(out_t)))
    torch.cuda.synchronize()
    log(f"serving: {len(items)} requests generated in {time.time() - t0:.1f}s")
    common = {"requests": len(items), "slots": args.serving_slots, "budget_gb": args.serving_budget_gb,
              "tol": 1e-8, "form": "fp32_refined"}
    budget = int(args.serving_budget_gb * (1 << 30))
    legs = {}
    with serve.Server(budget, slots=args.serving_slots) as srv:
        res = serve.replay(srv, items)
        legs["poisson"] = _serving_stats(srv.stats(), res, dict(common, rate_per_s=args.serving_rate))
    with serve.Server(budget, slots=args.serving_slots) as srv:
        res = serve.replay(srv, [dict(it, arrival_s=0.0) for it in items])
        legs["burst"] = _serving_stats(srv.stats(), res, dict(common, rate_per_s=None, arrivals="all at t=0"))
    log(f"serving: poisson {legs['poisson']}")
    log(f"serving: burst {legs['burst']}")

    # repeat leg: the first 32 cases, 8 requests each, round-robin order, Poisson arrivals
    ncase, per = min(32, len(items)), 8
    rng = np.random.default_rng(44)
    rep, rkeep = [], []
    arrivals = np.cumsum(rng.exponential(1.0 / args.serving_rate, size=ncase * per))
    for m in range(ncase * per):
        ci, rnd = m % ncase, m // ncase
        c = cases[ci]
        rho_t, rhs_t, out_t = keep[ci]
        if rnd > 0:   # u + 0.01 xi: a nearby right-hand side, as successive steps of one case
            du, dv, dw = W.sequence_velocity_perturbation(rnd, c.nx, c.ny, c.nz, seed=1000 + ci)
            rhs_t = ppsolve.divergence(g(c.u + 0.01 * du), g(c.v + 0.01 * dv), g(c.w + 0.01 * dw), c.h)
            out_t = torch.empty_like(rhs_t)
            rkeep.append((rhs_t, out_t))
        rep.append(dict(arrival_s=float(arrivals[m]), case_id=10_000 + ci, cfg=items[ci]["cfg"],
                        rho=vp(rho_t) if rnd == 0 else None, rhs=vp(rhs_t), p_out=vp(out_t)))
    torch.cuda.synchronize()
    with serve.Server(budget, slots=args.serving_slots) as srv:
        res = serve.replay(srv, rep)
        warm = [r["stats"]["inner_iters_total"] for r in res if r["status"] == 0 and not r["new_density"]]
        cold = [r["stats"]["inner_iters_total"] for r in res if r["status"] == 0 and r["new_density"]]
        legs["repeat"] = _serving_stats(srv.stats(), res, dict(
            common, requests=len(rep), cases=ncase, rate_per_s=args.serving_rate,
            resident_hits=len(warm), iters_median_first_request=int(np.median(cold)) if cold else None,
            iters_median_warm=int(np.median(warm)) if warm else None))
    log(f"serving: repeat {legs['repeat']}")
    out = dict(legs["poisson"], **{k: v for k, v in common.items()}, rate_per_s=args.serving_rate)
    out["legs"] = legs
    return out


def sequence_leg(args, log):
    """The moving-bubble time sequence: 192x192x384, 400 bubbles of 12 cells, each step a request
    of one resident case in the serving loop (new density, warm start), refined to 1e-10.
    Returns the summary and the last step's pressure and host inputs (checked against the oracle
    in the CPU-baseline leg)."""
    from paper_2104_01636_amd import sequence, workload as W

    case = W.preset("duct192")
    iters, step_ms, solve_ms, setup_ms = [], [], [], []
    t0 = time.time()
    last, sst = None, {}
    for s, p, st, item, srv in sequence.run(case, args.sequence_steps, mode="fp32_refined", tol=args.tol):
        iters.append(st["inner_iters_total"])
        step_ms.append(st["step_ms"])
        solve_ms.append(st["solve_ms"])
        setup_ms.append(st["setup_ms"])
        if s == args.sequence_steps - 1:
            last = (case, p.cpu().numpy(), item)
            sst = srv.stats()
    out = {"workload": f"{case.nx}x{case.ny}x{case.nz}, {len(case.centres)} bubbles d={case.diameter:g}, "
                       f"+0.5 cell per step", "steps": len(iters), "form": "fp32_refined", "tol": args.tol,
           "served": "one resident case, new density and warm start every step",
           "iters_first": iters[0], "iters_mean_after_first": round(float(np.mean(iters[1:])), 2) if len(iters) > 1 else None,
           "iters_max": max(iters), "step_ms_p50": round(pct(step_ms, 50), 2), "step_ms_p99": round(pct(step_ms, 99), 2),
           "solve_ms_p50": round(pct(solve_ms, 50), 2), "setup_ms_p50": round(pct(setup_ms, 50), 3),
           "evictions": sst.get("evictions"), "resident_cases": sst.get("resident_cases"),
           "wall_s": round(time.time() - t0, 1)}
    log(f"sequence: {out}")
    return out, last


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline_leg(args, case, results, seq_last, gpu_ms, log):
    """The float64 CPU oracle on the same (rho, b), on all host threads: its stencil-apply rate, its
    time to the same tolerance from a zero guess (its own MG-preconditioned CG, hierarchy set-up
    included), and its reference pressure (continued to 1e-13 from its own answer), against which
    every GPU result of this run is measured: L-infinity error and the oracle's residual per form,
    and the same for the last step of the served sequence."""
    from oracle import cref, poisson as P

    n = case.n_cells
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h)
    nthreads = cref.num_threads()
    x = np.random.default_rng(0).standard_normal(rho.shape)
    cref.apply_operator(rho, x, case.h)
    t = time.perf_counter()
    for _ in range(3):
        cref.apply_operator(rho, x, case.h)
    apply_s = (time.perf_counter() - t) / 3
    p1, it1, rr1, s1 = cref.solve(rho, b, case.h, tol=args.tol, maxit=4000)
    log(f"cpu baseline: oracle to {args.tol:g} in {s1:.1f} s, {it1} iterations, residual {rr1:.2e}, "
        f"{nthreads} threads")
    p_ref, it2, rr2, s2 = cref.solve(rho, b, case.h, tol=1e-13, maxit=4000, x0=p1)
    check = {}
    for m, r in results.items():
        check[m] = {"oracle_residual": float(f"{cref.relative_residual(rho, b, r['p'], case.h):.3e}"),
                    "linf_vs_oracle": float(f"{P.relative_linf_error(r['p'], p_ref):.3e}")}
        log(f"{m} vs oracle: {check[m]}")
    cpu = {"value": round(n * it1 / s1, 1), "unit": "cells*iters/s", "cores": nthreads, "kind": "oracle",
           "sample": f"the oracle's float64 solve of the same {case.nx}x{case.ny}x{case.nz} input (rho, b) to "
                     f"{args.tol:g} from a zero guess: {it1} iterations of its MG-preconditioned CG "
                     f"(damped-Jacobi V-cycle), {s1:.1f} s including its hierarchy set-up",
           "time_to_tol_s": round(s1, 3), "iters": it1, "rel_residual": float(f"{rr1:.3e}"),
           "stencil_apply_cells_per_s": round(n / apply_s, 1), "host_cpu": cpu_model(), "threads": nthreads,
           "gpu_time_to_tol_speedup": {m: round(s1 * 1e3 / ms, 1) for m, ms in gpu_ms.items()},
           "reference": {"tol": 1e-13, "extra_iters": it2, "rel_residual": float(f"{rr2:.3e}"),
                         "seconds": round(s2, 1)}}
    seq = None
    if seq_last is not None:
        scase, pn, item = seq_last
        rho_s = P.density_from_fraction(item[1])
        b_s = P.divergence(item[2], item[3], item[4], scase.h)
        pr, _, rr_s, _ = cref.solve(rho_s, b_s, scase.h, tol=1e-13)
        seq = {"last_step_oracle_residual": float(f"{cref.relative_residual(rho_s, b_s, pn, scase.h):.3e}"),
               "last_step_linf_vs_oracle": float(f"{P.relative_linf_error(pn, pr):.3e}")}
        log(f"sequence last step vs oracle: {seq}")
    return cpu, check, seq


def next_rows_leg(args, case, log, alpha_t, u_t, v_t, w_t, rho_t, rhs_t, p_t):
    """The steps on either side of the solve and the paper's own solver form, on the same input.

    * Time per call of the mixture density, the divergence (step 11's right-hand side), the face
      projection (step 12) and the surface-tension right-hand side (eq. ppe_surface_tension):
      torch events on the current stream, which is the stream the library launches them on,
      around repeated calls.  Each call ends by synchronising its stream, so the time per call
      includes one launch gap; the rates are algorithmic bytes (each array element read or
      written once) over that time, a lower bound on the kernel's own rate.
    * Multigrid as the solver (red-black SOR V- and W-cycles, no CG; Section 2.1) in float64, to
      the same tolerance from a zero guess, for SOR factors 1.0 and 1.15."""
    import torch
    from paper_2104_01636_amd import ppsolve

    n = case.n_cells
    reps = 10
    kappa_t = torch.full_like(alpha_t, 2.0 / (0.5 * case.diameter * case.h))  # curvature of a bubble
    out_t = torch.empty_like(alpha_t)
    u2, v2, w2 = u_t.clone(), v_t.clone(), w_t.clone()
    uc, vc, wc = u_t.clone(), v_t.clone(), w_t.clone()   # cell-centred velocity stand-ins
    calls = {  # name: (launch, algorithmic bytes per cell)
        "density_from_fraction": (lambda: ppsolve.density_from_fraction(alpha_t, 1000.0, 1.2, out=out_t), 16),
        "divergence": (lambda: ppsolve.divergence(u_t, v_t, w_t, case.h, 1.0, out=out_t), 32),
        "project": (lambda: ppsolve.project(rho_t, p_t, u2, v2, w2, case.h, 1e-3), 64),
        "surface_tension_rhs": (lambda: ppsolve.surface_tension_rhs(rho_t, alpha_t, kappa_t, 0.072, case.h,
                                                                    out=out_t), 32),
        # step 12 on faces and cells with the surface-tension pressure: reads rho, p, pt, three face and
        # three cell velocity components, writes the six velocity components
        "correct_velocity": (lambda: ppsolve.correct_velocity(rho_t, p_t, out_t, u2, v2, w2, uc, vc, wc, case.h,
                                                              1e-3), 120),
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
    del u2, v2, w2, uc, vc, wc, kappa_t, out_t

    mg = {}
    for cycle, omega in (("V", 1.0), ("V", 1.15), ("W", 1.0), ("W", 1.15)):
        flags = ppsolve.PP_FLAG_MG_SOLVER | (ppsolve.PP_FLAG_W_CYCLE if cycle == "W" else 0)
        with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=args.tol, max_iters=4000,
                            flags=flags, omega=omega) as S:
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
            mg[f"{cycle}_omega_{omega:g}"] = {"time_to_tol_ms": round(times[0], 3), "cycles": int(st["iters"]),
                                      "ms_per_cycle": round(st["solve_ms"] / max(1, st["iters"]), 4),
                                      "rel_residual": float(f"{st['rel_residual']:.3e}")}
            log(f"next rows: multigrid solver {cycle}-cycle omega {omega:g}: {times[0]:.1f} ms, {st['iters']} cycles, "
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
    ap.add_argument("--sequence-steps", type=int, default=200,
                    help="steps of the served moving-bubble sequence (192x192x384); 0 skips it")
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
        p_host = p_t.detach().cpu().numpy().copy()
        # the same steps once more with the Krylov steps replayed from HIP graphs (no per-kernel
        # events: the timed steps above launch directly so that every kernel can be bracketed)
        gtimes = []
        if args.kernel_timing == "timed":
            step(S)
            torch.cuda.synchronize()
            for _ in range(args.steps):
                a = time.perf_counter()
                step(S)
                torch.cuda.synchronize()
                gtimes.append((time.perf_counter() - a) * 1e3)
        iters = [st["inner_iters_total"] if mode == "fp32_refined" else st["iters"] for st in stats]
        results[mode] = dict(total_s=T1 - T0, times=times, stats=stats, iters=iters, kernels=kt, p=p_host,
                             graph_times=gtimes)
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

    seq, seq_last = None, None
    if args.sequence_steps > 0:
        seq, seq_last = sequence_leg(args, log)

    cpu, vs_oracle = None, None
    if not args.no_cpu_baseline:
        gpu_ms = {m: pct(results[m]["times"], 50) for m in results}
        cpu, vs_oracle, seq_check = cpu_baseline_leg(args, case, results, seq_last, gpu_ms, log)
        if seq is not None and seq_check is not None:
            seq.update(seq_check)

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
        "timed_steps": ("kernels launched directly with HIP events around every finest-level launch (graph "
                        "replay off), as the roofline needs; the same steps replayed from HIP graphs follow"),
        "time_to_tol_ms_graph_replay": {m: {"p50": round(pct(results[m]["graph_times"], 50), 3),
                                            "p99": round(pct(results[m]["graph_times"], 99), 3)}
                                        for m in results if results[m]["graph_times"]},
        "speedup_fp32_refined_vs_fp64": (round(pct(tt["fp64"], 50) / pct(tt["fp32_refined"], 50), 3)
                                         if "fp64" in tt and "fp32_refined" in tt else None),
        "iters": {m: {"krylov": int(np.median(results[m]["iters"])),
                      "outer": int(results[m]["stats"][0]["outer_iters"])} for m in results},
        "setup_ms": round(head["stats"][0]["setup_ms"], 3),
        "rel_residual": {m: float(f"{results[m]['stats'][-1]['rel_residual']:.3e}") for m in results},
        "linf_refined_vs_fp64": float(f"{diff_modes:.3e}") if diff_modes is not None else None,
        "vs_oracle": vs_oracle,
        "cells_per_s_solved": round(n / (ms_per_step * 1e-3), 1),
        "roofline": roof,
        "kernels": kern_tab,
        "next_rows": next_rows,
        "serving": serving,
        "sequence": seq,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
