"""The paper's solver form: multigrid cycles with red-black SOR as the solver (no CG).

Section 2.1 solves the pressure equations by red-black SOR relaxation
accelerated by multigrid; PP_FLAG_MG_SOLVER runs the library's V-cycle (red-black SOR smoothing with a
factor omega) as a stationary iteration x += M (bbar - A x), and with
PP_FLAG_W_CYCLE a W-cycle (every coarse level visited twice).  The answer must
be the same discrete solution: oracle residual and reference pressure.
"""
import numpy as np
import pytest
import torch

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, workload as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cycle", ["V", "W"])
@pytest.mark.parametrize("name", ["duct32", "duct128"])
@pytest.mark.parametrize("omega", [1.0, 1.15])
def test_multigrid_sor_solver_reaches_the_same_solution(name, omega, cycle):
    print("mg-solver", name, omega, cycle, flush=True)
    flags = ppsolve.PP_FLAG_MG_SOLVER | (ppsolve.PP_FLAG_W_CYCLE if cycle == "W" else 0)
    case = W.preset(name)
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
    rho_t = ppsolve.density_from_fraction(g(case.alpha))
    b_t = ppsolve.divergence(g(case.u), g(case.v), g(case.w), case.h)
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=1e-10, max_iters=3000,
                        flags=flags, omega=omega) as S:
        S.set_density(rho_t)
        p_t, st = S.solve(b_t)
    p = p_t.cpu().numpy()
    rr = cref.relative_residual(rho, b, p, case.h)
    print(f"   cycles {st['iters']}, oracle residual {rr:.2e}, {st['solve_ms']:.1f} ms", flush=True)
    assert rr <= 1e-10
    if name == "duct32":
        p_ref, *_ = cref.solve(rho, b, case.h, tol=1e-13)
        assert P.relative_linf_error(p, p_ref) < 1e-7


def test_flag_validation():
    with pytest.raises(ppsolve.PPError) as e:
        ppsolve.Solver(8, 8, 16, mode="fp32_refined", flags=ppsolve.PP_FLAG_MG_SOLVER)
    assert e.value.code == ppsolve.PP_ERR_INVALID
    with pytest.raises(ppsolve.PPError):
        ppsolve.Solver(8, 8, 16, omega=2.5)
    with pytest.raises(ppsolve.PPError) as e:    # W-cycles only in the multigrid-solver form
        ppsolve.Solver(8, 8, 16, flags=ppsolve.PP_FLAG_W_CYCLE)
    assert e.value.code == ppsolve.PP_ERR_INVALID
