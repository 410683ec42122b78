"""Time sequence with moving bubbles: warm-started solves against the oracle.

Full-size 192x192x384 (400 bubbles of 12 cells) for a few steps, accepted by
the oracle's residual at every step; and a 64x64x128 sequence whose last
pressure is compared with the oracle's reference solution (drift).
"""
import json
import os

import numpy as np
import pytest

from oracle import cref, poisson as P
from paper_2104_01636_amd import sequence, workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def oracle_inputs(item, h):
    s, alpha, u, v, w = item
    return P.density_from_fraction(alpha), P.divergence(u, v, w, h)


@pytest.mark.parametrize("mode", ["fp32_refined", "fp64"])
def test_sequence_192_warm_start(mode):
    case = W.preset("duct192")
    say("sequence 192x192x384", mode)
    iters = []
    for s, p, st, item in sequence.run(case, 6, mode=mode, tol=1e-10):
        rho, b = oracle_inputs(item, case.h)
        pn = p.cpu().numpy()
        rr = cref.relative_residual(rho, b, pn, case.h)
        it = st["inner_iters_total"] if mode == "fp32_refined" else st["iters"]
        iters.append(it)
        say(f"   step {s}: iters {it} outer {st['outer_iters']} oracle residual {rr:.2e} step {st['step_ms']:.1f} ms")
        assert rr <= 1e-10
        assert abs(pn.mean()) <= 1e-12 * np.abs(pn).max()
    # Moving every interface by half a cell changes the operator a lot near the bubbles, so a
    # warm start saves few iterations here; the count must stay of the cold step's order.
    assert max(iters) <= 2 * iters[0]


def test_sequence_drift_against_reference():
    case = W.make_case(64, 64, 128, 24, 8.0, seed=15)
    say("sequence 64x64x128 drift")
    last = None
    for s, p, st, item in sequence.run(case, 10, mode="fp32_refined", tol=1e-10):
        rho, b = oracle_inputs(item, case.h)
        last = (p.cpu().numpy(), rho, b)
        assert cref.relative_residual(rho, b, last[0], case.h) <= 1e-10
    p, rho, b = last
    p_ref, it, rr, _ = cref.solve(rho, b, case.h, tol=1e-13)
    err = P.relative_linf_error(p, p_ref)
    say(f"   drift after 10 steps: L-inf {err:.2e} (oracle {it} iterations, residual {rr:.1e})")
    assert err < 1e-7


@pytest.mark.skipif(os.environ.get("PP_FULL_SEQUENCE") != "1", reason="200-step run (set PP_FULL_SEQUENCE=1)")
@pytest.mark.timeout(1200)
def test_sequence_192_full_200_steps():
    """The full time sequence: 200 steps on 192x192x384 (400 bubbles of 12 cells moving
    +0.5 cell in z per step with lateral jitter), warm-started, float32-refined to 1e-10.
    Every step is accepted by the oracle's residual; every 20th step is compared with the
    oracle's reference pressure (L-inf drift)."""
    case = W.preset("duct192")
    iters, times, drift = [], [], []
    for s, p, st, item in sequence.run(case, 200, mode="fp32_refined", tol=1e-10):
        rho, b = oracle_inputs(item, case.h)
        pn = p.cpu().numpy()
        rr = cref.relative_residual(rho, b, pn, case.h)
        iters.append(st["inner_iters_total"])
        times.append(st["step_ms"])
        line = {"step": s, "iters": iters[-1], "oracle_residual": float(f"{rr:.3e}"), "step_ms": round(st["step_ms"], 2)}
        if s % 20 == 0 or s == 199:
            p_ref, _, rr_ref, _ = cref.solve(rho, b, case.h, tol=1e-13)
            drift.append(P.relative_linf_error(pn, p_ref))
            line["linf_vs_reference"] = float(f"{drift[-1]:.3e}")
        say(json.dumps(line))
        assert rr <= 1e-10
    say(json.dumps({"summary": True, "steps": len(iters), "iters_first": iters[0],
                    "iters_mean_after_first": round(float(np.mean(iters[1:])), 2), "iters_max": max(iters),
                    "step_ms_median": round(float(np.median(times)), 2), "linf_max": float(f"{max(drift):.3e}")}))
    assert max(drift) < 1e-7
