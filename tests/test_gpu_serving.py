"""Serving loop on the GPU: results alone vs in the mix, admission, Poisson replay.

Requests follow the serving workload's recipe (grids from 32x32x64 to
128x128x256, 4-200 bubbles of 6-16 cells, refined float32/float64 solves to a
relative residual of 1e-8), with fewer requests than the full 256 so the test
stays short.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, serve, workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-8


def say(*a):
    print(*a, flush=True)


def build_requests(n, seed=4, rate=40.0):
    reqs = W.serving_requests(n, rate_hz=rate, seed=seed)
    items = []
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)  # noqa: E731
    for r in reqs:
        nx, ny, nz = r["grid"]
        c = W.make_case(nx, ny, nz, r["n_bubbles"], r["diameter"], seed=r["seed"])
        rho_t = ppsolve.density_from_fraction(g(c.alpha))
        rhs_t = ppsolve.divergence(g(c.u), g(c.v), g(c.w), c.h)
        items.append(dict(req=r, case=c, rho_t=rho_t, rhs_t=rhs_t,
                          cfg=ppsolve.make_config(nx, ny, nz, c.h, "fp32_refined", TOL)))
    torch.cuda.synchronize()
    return items


def solve_alone(it):
    c = it["case"]
    with ppsolve.Solver(c.nx, c.ny, c.nz, c.h, mode="fp32_refined", tol=TOL) as S:
        S.set_density(it["rho_t"])
        p, st = S.solve(it["rhs_t"])
    torch.cuda.synchronize()
    return p.cpu().numpy(), st


def vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


@pytest.fixture(scope="module")
def items():
    say("building serving requests")
    its = build_requests(16)
    for it in its:
        it["alone"], it["alone_stats"] = solve_alone(it)
    return its


def test_burst_results_identical_alone_and_in_the_mix(items):
    say("burst: all requests at t=0 on 4 slots")
    outs = [torch.empty_like(it["rhs_t"]) for it in items]
    with serve.Server(64 << 30, slots=4) as srv:
        ids = [srv.submit(i, it["cfg"], vp(it["rho_t"]), vp(it["rhs_t"]), vp(o)) for i, (it, o) in
               enumerate(zip(items, outs))]
        res = [srv.wait(r) for r in ids]
        st = srv.stats()
    say("   stats", st)
    assert all(r["status"] == 0 for r in res), [r["message"] for r in res if r["status"]]
    assert st["max_running"] >= 2
    for it, o in zip(items, outs):
        p = o.cpu().numpy()
        np.testing.assert_array_equal(p, it["alone"])
        rho = P.density_from_fraction(it["case"].alpha)
        b = P.divergence(it["case"].u, it["case"].v, it["case"].w, it["case"].h)
        assert cref.relative_residual(rho, b, p, it["case"].h) <= TOL


def test_small_budget_admission_and_eviction(items):
    say("small budget")
    fps = [ppsolve.footprint_bytes(it["case"].nx, it["case"].ny, it["case"].nz, "fp32_refined") for it in items]
    budget = int(2.2 * max(fps)) + (64 << 20)
    outs = [torch.empty_like(it["rhs_t"]) for it in items]
    with serve.Server(budget, slots=3) as srv:
        ids = [srv.submit(100 + i, it["cfg"], vp(it["rho_t"]), vp(it["rhs_t"]), vp(o))
               for i, (it, o) in enumerate(zip(items, outs))]
        res = [srv.wait(r) for r in ids]
        st = srv.stats()
    say("   stats", st)
    assert all(r["status"] == 0 for r in res)
    assert st["peak_resident_bytes"] <= budget and st["evictions"] > 0
    for it, o in zip(items, outs):
        np.testing.assert_array_equal(o.cpu().numpy(), it["alone"])


def test_poisson_replay_and_warm_resident_case(items):
    say("poisson replay at 40 req/s")
    outs = [torch.empty_like(it["rhs_t"]) for it in items]
    reqs = [dict(arrival_s=it["req"]["arrival_s"], case_id=200 + i, cfg=it["cfg"], rho=vp(it["rho_t"]),
                 rhs=vp(it["rhs_t"]), p_out=vp(o)) for i, (it, o) in enumerate(zip(items, outs))]
    with serve.Server(64 << 30, slots=4) as srv:
        res = serve.replay(srv, reqs)
        st = srv.stats()
        say("   stats", st)
        assert all(r["status"] == 0 for r in res)
        assert st["latency_p99_ms"] >= st["latency_p50_ms"] > 0 and st["solves_per_s"] > 0
        for it, o in zip(items, outs):
            np.testing.assert_array_equal(o.cpu().numpy(), it["alone"])
        # the same case again without a density: resident hierarchy, warm start from its pressure
        it = items[0]
        again = torch.empty_like(it["rhs_t"])
        r2 = srv.wait(srv.submit(200, it["cfg"], None, vp(it["rhs_t"]), vp(again)))
        assert r2["status"] == 0 and not r2["new_density"]
        assert r2["stats"]["iters"] == 0
        assert P.relative_linf_error(again.cpu().numpy(), it["alone"]) < 1e-12


def test_allocation_failure_is_reported(items, monkeypatch):
    """A device allocation failure at handle creation, forced from the host through
    PP_FAULT_OOM_AT (read when a handle is made), is an error status for the binding
    and for a serving request, and leaves nothing behind: the same request succeeds
    once the switch is gone."""
    it = items[0]
    c = it["case"]
    monkeypatch.setenv("PP_FAULT_OOM_AT", "1")
    with pytest.raises(ppsolve.PPError) as e:
        ppsolve.Solver(c.nx, c.ny, c.nz, c.h, mode="fp32_refined", tol=TOL)
    assert e.value.code == ppsolve.PP_ERR_OOM
    out = torch.zeros_like(it["rhs_t"])
    with serve.Server(64 << 30, slots=2) as srv:
        r = srv.wait(srv.submit(300, it["cfg"], vp(it["rho_t"]), vp(it["rhs_t"]), vp(out)))
        say("   forced failure", r["status"], r["message"])
        assert r["status"] == ppsolve.PP_ERR_OOM and "injected" in r["message"]
        monkeypatch.delenv("PP_FAULT_OOM_AT")
        r = srv.wait(srv.submit(300, it["cfg"], vp(it["rho_t"]), vp(it["rhs_t"]), vp(out)))
        st = srv.stats()
    say("   stats", st)
    assert r["status"] == 0
    assert st["rejected"] == 1 and st["succeeded"] == 1
    np.testing.assert_array_equal(out.cpu().numpy(), it["alone"])
