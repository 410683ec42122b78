"""pp_rel_residual (the acceptance measure of a solve taken on the device)
against the oracle's residual checker, on the same seeded inputs (needs an MI355X).

Tolerances: on iterates far from converged both sides compute the same O(1)
ratio, each with rounding of about 1e-16 per term: 1e-12 relative.  On a
converged pressure the residual is a cancellation of terms of the size of
bbar, so each side's absolute error in the ratio is about 1e-15: 1e-13
absolute (the ratio itself is about 1e-10 there).
"""
import numpy as np
import pytest
import torch

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


@pytest.mark.parametrize("shape", [(2, 2, 2), (4, 5, 3), (9, 7, 70), (34, 17, 10), (64, 32, 32)])
def test_rel_residual_matches_oracle_on_random_iterates(shape):
    nz, ny, nx = shape
    say("rel_residual", shape)
    case = W.random_small_case(300 + sum(shape), nx, ny, nz)
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h) + 0.25   # a mean to remove
    rng = np.random.default_rng(sum(shape))
    for scale in (1e-3, 1.0, 1e3):
        p = rng.standard_normal(shape) * scale
        ref = cref.relative_residual(rho, b, p, case.h)
        got = ppsolve.rel_residual(gpu(rho), gpu(b), gpu(p), case.h)
        assert got == pytest.approx(ref, rel=1e-12)
        assert ppsolve.rel_residual(gpu(rho), gpu(b), gpu(p), case.h) == got   # bitwise repeatable


def test_rel_residual_of_converged_solves():
    for name in ("duct32", "duct128"):
        case = W.preset(name)
        rho = P.density_from_fraction(case.alpha)
        b = P.divergence(case.u, case.v, case.w, case.h)
        with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=1e-10) as S:
            S.set_density(gpu(rho))
            p_t, st = S.solve(gpu(b))
        ref = cref.relative_residual(rho, b, p_t.cpu().numpy(), case.h)
        got = ppsolve.rel_residual(gpu(rho), gpu(b), p_t, case.h)
        say(name, "oracle", ref, "device", got, "solver", st["rel_residual"])
        assert abs(got - ref) <= 1e-13 and got <= 1e-10


def test_rel_residual_edge_cases():
    nz, ny, nx = 4, 3, 5
    rho = gpu(np.full((nz, ny, nx), 2.0))
    zero = torch.zeros((nz, ny, nx), dtype=torch.float64, device=DEV)
    # constant right-hand side: bbar = 0; zero residual for p = const, infinite otherwise
    assert ppsolve.rel_residual(rho, zero + 3.0, zero + 1.0, 0.5) == 0.0
    p = zero.clone()
    p[1, 1, 1] = 1.0
    assert ppsolve.rel_residual(rho, zero + 3.0, p, 0.5) == float("inf")
    bad = rho.clone()
    bad[0, 0, 0] = 0.0
    with pytest.raises(ppsolve.PPError) as e:
        ppsolve.rel_residual(bad, zero, zero, 0.5)
    assert e.value.code == ppsolve.PP_ERR_NONFINITE
    b2 = zero.clone()
    b2[2, 2, 2] = float("nan")
    with pytest.raises(ppsolve.PPError) as e:
        ppsolve.rel_residual(rho, b2, zero, 0.5)
    assert e.value.code == ppsolve.PP_ERR_NONFINITE
    with pytest.raises(ppsolve.PPError) as e:
        ppsolve.rel_residual(rho, zero, zero, 0.0)
    assert e.value.code == ppsolve.PP_ERR_INVALID
