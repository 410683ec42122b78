"""The serving scheduler (pp_server, C++) driven by a host backend: no GPU needed.

The fake backend keeps each case's density and last pressure in host memory
and solves with the CPU oracle, so admission, residency, eviction, warm starts,
concurrency, statistics and error propagation are checked against the
oracle's answers.
"""
import ctypes
import threading
import time

import numpy as np
import pytest

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, serve, workload as W


class FakeBackend:
    """Host implementation of the pp_backend table."""

    def __init__(self, bytes_per_cell=64, delay_s=0.0, fail_open=()):
        self.bpc = bytes_per_cell
        self.delay = delay_s
        self.fail_open = set(fail_open)
        self.cases = {}
        self.next = 1
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.opened = 0
        self.closed = 0
        self.errors = {}
        self._msg = ctypes.create_string_buffer(160)
        self.table = serve.Backend(
            None,
            serve.FOOTPRINT_FN(self._footprint),
            serve.OPEN_FN(self._open),
            serve.SETRHO_FN(self._set_density),
            serve.SOLVE_FN(self._solve),
            serve.CLOSE_FN(self._close),
            serve.ERROR_FN(self._error),
        )

    def _footprint(self, ctx, cfgp):
        c = cfgp.contents
        if c.nz % 2 or c.nx < 2:
            return 0
        return c.nx * c.ny * c.nz * self.bpc

    def _open(self, ctx, cfgp, out):
        c = cfgp.contents
        if (c.nx, c.ny, c.nz) in self.fail_open:
            self.errors[0] = b"injected allocation failure"
            return ppsolve.PP_ERR_OOM
        with self.lock:
            key = self.next
            self.next += 1
            self.opened += 1
        shape = (c.nz, c.ny, c.nx)
        self.cases[key] = {"shape": shape, "h": c.h, "tol": c.tol, "rho": None, "p": np.zeros(shape)}
        out[0] = key
        return 0

    def _arr(self, ptr, shape):
        n = int(np.prod(shape))
        return np.ctypeslib.as_array((ctypes.c_double * n).from_address(ptr)).reshape(shape)

    def _set_density(self, ctx, cs, rho):
        cs = self.cases[cs]
        cs["rho"] = self._arr(rho, cs["shape"]).copy()
        return 0

    def _solve(self, ctx, key, rhs, p_out, st):
        cs = self.cases[key]
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
        try:
            time.sleep(self.delay)
            b = self._arr(rhs, cs["shape"]).copy()
            p, it, rr, _ = cref.solve(cs["rho"], b, cs["h"], tol=cs["tol"], x0=cs["p"])
            cs["p"] = p
            if p_out:
                self._arr(p_out, cs["shape"])[...] = p
            st.contents.iters = it
            st.contents.rel_residual = rr
            return 0
        finally:
            with self.lock:
                self.active -= 1

    def _close(self, ctx, key):
        self.cases.pop(key, None)
        self.closed += 1

    def _error(self, ctx, key):
        self._msg.value = self.errors.get(0, b"fake backend error")
        return ctypes.addressof(self._msg)


def cfg_of(case, tol=1e-10):
    return ppsolve.make_config(case.nx, case.ny, case.nz, case.h, "fp64", tol)


def make_inputs(case):
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h)
    return rho, b


def ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def test_results_alone_and_in_the_mix_are_identical():
    cases = [W.make_case(8 * s, 8 * s, 16 * s, 3, 4.0, seed=40 + s) for s in (1, 2, 1, 3, 2)]
    inputs = [make_inputs(c) for c in cases]
    # alone: one request at a time
    fb = FakeBackend()
    alone = []
    with serve.Server(1 << 40, slots=1, backend=fb.table) as srv:
        for i, (c, (rho, b)) in enumerate(zip(cases, inputs)):
            out = np.zeros(c.shape)
            rid = srv.submit(100 + i, cfg_of(c), ptr(rho), ptr(b), ptr(out))
            res = srv.wait(rid)
            assert res["status"] == 0
            alone.append(out)
    # in the mix: all at once on three slots
    fb2 = FakeBackend(delay_s=0.05)
    outs = [np.zeros(c.shape) for c in cases]
    with serve.Server(1 << 40, slots=3, backend=fb2.table) as srv:
        ids = [srv.submit(100 + i, cfg_of(c), ptr(rho), ptr(b), ptr(o))
               for i, (c, (rho, b), o) in enumerate(zip(cases, inputs, outs))]
        res = [srv.wait(r) for r in ids]
        st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert fb2.max_active >= 2 and st["max_running"] >= 2
    for a, b_, c, (rho, b) in zip(alone, outs, cases, inputs):
        # the host oracle's OpenMP reductions change order with the thread-team size of
        # concurrent callers, so alone and mixed agree to rounding here (bitwise on the GPU)
        assert P.relative_linf_error(a, b_) < 1e-11
        assert cref.relative_residual(rho, b, b_, c.h) <= 1e-10
    assert st["succeeded"] == len(cases) and st["latency_p99_ms"] >= st["latency_p50_ms"] > 0
    assert st["solves_per_s"] > 0


def test_admission_by_footprint_and_lru_eviction():
    cases = [W.make_case(8, 8, 16, 2, 4.0, seed=60 + i) for i in range(6)]
    inputs = [make_inputs(c) for c in cases]
    fb = FakeBackend(bytes_per_cell=64)
    one = 8 * 8 * 16 * 64
    with serve.Server(2 * one + one // 2, slots=2, backend=fb.table) as srv:
        ids = []
        for i, (c, (rho, b)) in enumerate(zip(cases, inputs)):
            ids.append(srv.submit(i, cfg_of(c), ptr(rho), ptr(b), None))
        res = [srv.wait(r) for r in ids]
        st = srv.stats()
        assert all(r["status"] == 0 for r in res)
        assert st["peak_resident_bytes"] <= 2 * one + one // 2
        assert st["resident_cases"] <= 2 and st["evictions"] >= 4
        # a case larger than the whole budget is rejected, the server keeps going
        big = W.make_case(16, 16, 32, 2, 4.0, seed=70)
        rho, b = make_inputs(big)
        rid = srv.submit(99, cfg_of(big), ptr(rho), ptr(b), None)
        assert srv.wait(rid)["status"] == ppsolve.PP_ERR_OOM
        c, (rho, b) = cases[0], inputs[0]
        rid = srv.submit(0, cfg_of(c), ptr(rho), ptr(b), None)
        assert srv.wait(rid)["status"] == 0
    assert fb.opened == fb.closed


def test_warm_start_residency_and_state_errors():
    case = W.make_case(16, 16, 32, 3, 5.0, seed=80)
    rho, b = make_inputs(case)
    fb = FakeBackend()
    with serve.Server(1 << 40, slots=2, backend=fb.table) as srv:
        # the first request of a case must bring a density
        rid = srv.submit(7, cfg_of(case), None, ptr(b), None)
        r = srv.wait(rid)
        assert r["status"] == ppsolve.PP_ERR_STATE
        out = np.zeros(case.shape)
        r1 = srv.wait(srv.submit(7, cfg_of(case), ptr(rho), ptr(b), ptr(out)))
        assert r1["status"] == 0 and r1["new_density"] and r1["stats"]["iters"] > 0
        # same right-hand side again, density kept resident: warm start converges at once
        r2 = srv.wait(srv.submit(7, cfg_of(case), None, ptr(b), ptr(out)))
        assert r2["status"] == 0 and not r2["new_density"] and r2["stats"]["iters"] == 0
        # a request with a different grid for an existing case is invalid
        other = ppsolve.make_config(8, 8, 16)
        r3 = srv.wait(srv.submit(7, other, ptr(rho), ptr(b), None))
        assert r3["status"] == ppsolve.PP_ERR_INVALID


def test_injected_open_failure_does_not_lose_other_cases():
    good = [W.make_case(8, 8, 16, 2, 4.0, seed=90 + i) for i in range(3)]
    bad = W.make_case(12, 12, 16, 2, 4.0, seed=95)
    fb = FakeBackend(fail_open={(12, 12, 16)})
    with serve.Server(1 << 40, slots=2, backend=fb.table) as srv:
        ids = []
        for i, c in enumerate(good[:2] + [bad] + good[2:]):
            rho, b = make_inputs(c)
            c._keep = (rho, b)
            ids.append(srv.submit(i, cfg_of(c), ptr(rho), ptr(b), None))
        res = [srv.wait(r) for r in ids]
    assert [r["status"] for r in res] == [0, 0, ppsolve.PP_ERR_OOM, 0]
    assert "injected" in res[2]["message"]
    assert fb.opened == 3


def test_replay_timestamps_follow_arrivals():
    reqs = W.serving_requests(12, rate_hz=200.0, seed=4, grids=((8, 8, 16), (16, 16, 32)))
    fb = FakeBackend()
    keep = []
    items = []
    for r in reqs:
        nx, ny, nz = r["grid"]
        c = W.make_case(nx, ny, nz, min(r["n_bubbles"], 2), min(r["diameter"], 4.0), seed=r["seed"])
        rho, b = make_inputs(c)
        keep.append((rho, b))
        items.append(dict(arrival_s=r["arrival_s"], case_id=r["index"], cfg=cfg_of(c), rho=ptr(rho), rhs=ptr(b),
                          p_out=None))
    with serve.Server(1 << 40, slots=3, backend=fb.table) as srv:
        res = serve.replay(srv, items)
    subs = np.array([r["t_submit"] for r in res])
    arr = np.array([r["arrival_s"] for r in reqs])
    assert np.all(np.diff(subs) >= 0)
    np.testing.assert_allclose(subs - subs[0], arr - arr[0], atol=0.05)
    assert all(r["status"] == 0 for r in res)
