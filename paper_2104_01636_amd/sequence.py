"""Time sequence of pressure solves with moving bubbles, served warm-started.

Each step moves every bubble +0.5 cell along z plus a seeded lateral jitter,
recomputes the gas fraction, perturbs the face velocities (u_s = u_0 + 0.01 xi_s
with seeded U[-1, 1] xi_s), and hands the step's density and right-hand side to
the serving loop (include/pp_server.h) as a request of one resident case: the
case's solver handle, hierarchy and last pressure stay on the device between
steps, the set-up reruns for the new density, and every solve starts from the
previous step's pressure.  Inputs for the next steps are generated on host
threads while the GPU solves the current one.

    python -m paper_2104_01636_amd.sequence --steps 200      # one JSON line per step
"""
from __future__ import annotations

import argparse
import ctypes
import json
import queue
import sys
import threading
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import ppsolve, serve, workload as W


def host_steps(case: W.Case, steps: int, seed: int = 5, eps: float = 0.01, workers: int = 4):
    """Yields (step, alpha, u, v, w) on the host, in step order; steps are made on
    `workers` threads, at most 2 * workers ahead of the consumer."""
    centres = list(W.moving_sequence(case, steps, seed=seed))

    def make(sc):
        s, c = sc
        alpha = W.volume_fraction(case.nx, case.ny, case.nz, c, case.diameter)
        du, dv, dw = W.sequence_velocity_perturbation(s, case.nx, case.ny, case.nz, seed=seed)
        return s, alpha, case.u + eps * du, case.v + eps * dv, case.w + eps * dw

    ahead = 2 * max(1, workers)
    with ThreadPoolExecutor(max(1, workers)) as ex:
        futs = [ex.submit(make, sc) for sc in centres[:ahead]]
        nxt = len(futs)
        for i in range(len(centres)):
            item = futs[i].result()
            futs[i] = None
            if nxt < len(centres):
                futs.append(ex.submit(make, centres[nxt]))
                nxt += 1
            yield item


def run(case: W.Case, steps: int, mode: str = "fp32_refined", tol: float = 1e-10, seed: int = 5, device="cuda:0",
        prefetch: int = 2, workers: int = 4, case_id: int = 0):
    """Serve the sequence as requests of one resident case; yields
    (step, p_tensor, stats, host_inputs, server) per step.

    stats is the request's pp_stats plus step_ms (density, divergence and the
    request from submit to result), latency_ms (the request alone) and
    new_density.  p_tensor receives the step's pressure (overwritten by the next
    step: copy it to keep it).  server is the serving loop (its stats show the
    case resident)."""
    import torch

    q: queue.Queue = queue.Queue(maxsize=prefetch)

    def producer():
        try:
            for item in host_steps(case, steps, seed, workers=workers):
                q.put(item)
        finally:
            q.put(None)

    th = threading.Thread(target=producer, daemon=True)
    th.start()
    dev = torch.device(device)
    p = torch.zeros((case.nz, case.ny, case.nx), dtype=torch.float64, device=dev)
    rho = torch.empty_like(p)
    rhs = torch.empty_like(p)
    cfg = ppsolve.make_config(case.nx, case.ny, case.nz, case.h, mode, tol, 4000)
    need = ppsolve.footprint_bytes(case.nx, case.ny, case.nz, mode) + 8 * case.n_cells
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    with serve.Server(2 * need + (64 << 20), slots=1) as srv:
        while True:
            item = q.get()
            if item is None:
                break
            s, alpha, u, v, w = item
            a_t = torch.from_numpy(alpha).to(dev)
            u_t, v_t, w_t = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (u, v, w))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ppsolve.density_from_fraction(a_t, out=rho)
            ppsolve.divergence(u_t, v_t, w_t, case.h, out=rhs)
            torch.cuda.synchronize()  # the case runs on its own stream
            rid = srv.submit(case_id, cfg, vp(rho), vp(rhs), vp(p))
            res = srv.wait(rid)
            if res["status"] != 0:
                raise ppsolve.PPError(res["status"], f"step {s}: {res['message']}")
            st = dict(res["stats"])
            st["step_ms"] = (time.perf_counter() - t0) * 1e3
            st["latency_ms"] = res["latency_ms"]
            st["new_density"] = res["new_density"]
            yield s, p, st, item, srv
    th.join()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--workload", default="duct192")
    ap.add_argument("--mode", default="fp32_refined")
    ap.add_argument("--tol", type=float, default=1e-10)
    args = ap.parse_args(argv)
    case = W.preset(args.workload)
    iters = []
    for s, p, st, _, _ in run(case, args.steps, args.mode, args.tol):
        iters.append(st["inner_iters_total"] if args.mode == "fp32_refined" else st["iters"])
        print(json.dumps({"step": s, "iters": iters[-1], "outer": st["outer_iters"], "rel_residual": st["rel_residual"],
                          "setup_ms": round(st["setup_ms"], 3), "solve_ms": round(st["solve_ms"], 3),
                          "step_ms": round(st["step_ms"], 3)}), flush=True)
    print(json.dumps({"summary": True, "steps": len(iters), "iters_first": iters[0] if iters else None,
                      "iters_mean_after_first": float(np.mean(iters[1:])) if len(iters) > 1 else None}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
