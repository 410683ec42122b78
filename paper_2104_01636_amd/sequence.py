"""Time sequence of pressure solves with moving bubbles, warm-started.

Each step moves every bubble +0.5 cell along z plus a seeded lateral jitter,
recomputes the gas fraction, perturbs the face velocities (u_s = u_0 + 0.01 xi_s
with seeded U[-1, 1] xi_s), and solves on the GPU from the previous step's
pressure.  Inputs for the next step are generated on a host thread while the
GPU solves the current one.

    python -m paper_2104_01636_amd.sequence --steps 200      # one JSON line per step
"""
from __future__ import annotations

import argparse
import json
import queue
import sys
import threading
import time

import numpy as np

from . import ppsolve, workload as W


def host_steps(case: W.Case, steps: int, seed: int = 5, eps: float = 0.01):
    """Yields (step, alpha, u, v, w) on the host."""
    for s, centres in W.moving_sequence(case, steps, seed=seed):
        alpha = W.volume_fraction(case.nx, case.ny, case.nz, centres, case.diameter)
        du, dv, dw = W.sequence_velocity_perturbation(s, case.nx, case.ny, case.nz, seed=seed)
        yield s, alpha, case.u + eps * du, case.v + eps * dv, case.w + eps * dw


def run(case: W.Case, steps: int, mode: str = "fp32_refined", tol: float = 1e-10, seed: int = 5, device="cuda:0",
        prefetch: int = 2):
    """Solve the sequence; yields (step, p_tensor, stats, host_inputs) per step.

    p_tensor is the solver's resident pressure (overwritten by the next step:
    copy it to keep it)."""
    import torch

    q: queue.Queue = queue.Queue(maxsize=prefetch)

    def producer():
        for item in host_steps(case, steps, seed):
            q.put(item)
        q.put(None)

    th = threading.Thread(target=producer, daemon=True)
    th.start()
    dev = torch.device(device)
    p = torch.zeros((case.nz, case.ny, case.nx), dtype=torch.float64, device=dev)
    rho = torch.empty_like(p)
    rhs = torch.empty_like(p)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=tol, max_iters=4000) as S:
        while True:
            item = q.get()
            if item is None:
                break
            s, alpha, u, v, w = item
            a_t = torch.from_numpy(alpha).to(dev)
            u_t, v_t, w_t = (torch.from_numpy(np.ascontiguousarray(x)).to(dev) for x in (u, v, w))
            t0 = time.perf_counter()
            ppsolve.density_from_fraction(a_t, out=rho)
            ppsolve.divergence(u_t, v_t, w_t, case.h, out=rhs)
            S.set_density(rho)
            _, st = S.solve(rhs, p)
            st["step_ms"] = (time.perf_counter() - t0) * 1e3
            yield s, p, st, item
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
    for s, p, st, _ in run(case, args.steps, args.mode, args.tol):
        iters.append(st["inner_iters_total"] if args.mode == "fp32_refined" else st["iters"])
        print(json.dumps({"step": s, "iters": iters[-1], "outer": st["outer_iters"], "rel_residual": st["rel_residual"],
                          "setup_ms": round(st["setup_ms"], 3), "solve_ms": round(st["solve_ms"], 3),
                          "step_ms": round(st["step_ms"], 3)}), flush=True)
    print(json.dumps({"summary": True, "steps": len(iters), "iters_first": iters[0] if iters else None,
                      "iters_mean_after_first": float(np.mean(iters[1:])) if len(iters) > 1 else None}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
