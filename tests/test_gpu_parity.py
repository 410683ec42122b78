"""GPU path vs the CPU oracle, through the C ABI (needs an MI355X).

Tolerances (float64 rounding of a 7-point stencil with 833:1 coefficient jumps):
  * density from fraction: bit-exact (same expression, no contraction);
  * divergence: bit-exact (same operation order);
  * operator A x: |A_gpu x - A_ref x| <= 1e-13 * max_c sum_f |beta_f (x_nb - x_c)| / h^2;
  * solves: relative residual computed by the oracle's own operator <= tol
    (1e-10 float64, 1e-10 refined unless stated), pressure error vs the oracle's
    reference solution (solved to 1e-13) < 1e-7 relative in L-infinity.
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


def cpu(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def inputs(case):
    """The same seeded (rho, b) on both sides: each side applies its own density
    rule and divergence to the generator's gas fraction and face velocities."""
    rho_ref = P.density_from_fraction(case.alpha)
    b_ref = P.divergence(case.u, case.v, case.w, case.h)
    rho_t = ppsolve.density_from_fraction(gpu(case.alpha))
    b_t = ppsolve.divergence(gpu(case.u), gpu(case.v), gpu(case.w), case.h)
    return rho_ref, b_ref, rho_t, b_t


SHAPES = [(2, 2, 2), (3, 5, 4), (7, 6, 8), (16, 8, 8), (33, 17, 10), (64, 32, 32)]  # (nz, ny, nx)
EVEN = [(2, 2, 2), (4, 5, 3), (6, 6, 8), (16, 8, 8), (34, 17, 10), (64, 32, 32),   # solver grids: nz even;
        (6, 10, 192), (4, 9, 128), (2, 3, 64),   # rows of 64-256 cells: the row-wave operator, ragged bands
        (6, 7, 256)]                             # (rows of 128 and 256 cells: each over two wavefronts)


@pytest.mark.parametrize("shape", SHAPES)
def test_density_and_divergence_bit_exact(shape):
    nz, ny, nx = shape
    say("density/divergence", shape)
    case = W.random_small_case(sum(shape), nx, ny, nz)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    np.testing.assert_array_equal(cpu(rho_t), rho_ref)
    np.testing.assert_array_equal(cpu(b_t), b_ref)
    b2 = ppsolve.divergence(gpu(case.u), gpu(case.v), gpu(case.w), case.h, dt=0.37)
    np.testing.assert_array_equal(cpu(b2), P.divergence(case.u, case.v, case.w, case.h, 0.37))


def op_scale(rho, x, h):
    bx, by, bz = P.face_coefficients(rho)
    s = np.zeros_like(x)
    s[:, :, :-1] += np.abs(bx[:, :, :-1] * (x[:, :, 1:] - x[:, :, :-1]))
    s[:, :-1, :] += np.abs(by[:, :-1, :] * (x[:, 1:, :] - x[:, :-1, :]))
    s += np.abs(bz * (np.roll(x, -1, 0) - x))
    return 2 * s.max() / h ** 2


@pytest.mark.parametrize("shape", EVEN + [(512, 256, 256)])
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_operator_matches_oracle(shape, mode):
    nz, ny, nx = shape
    say("apply", shape, mode)
    if shape == (512, 256, 256):
        case = W.preset("duct256")
    else:
        case = W.random_small_case(3 + sum(shape), nx, ny, nz)
    rho = P.density_from_fraction(case.alpha)
    x = np.random.default_rng(1).standard_normal(shape)
    with ppsolve.Solver(nx, ny, nz, case.h, mode=mode) as S:
        S.set_density(gpu(rho))
        y = cpu(S.apply(gpu(x)))
    ref = cref.apply_operator(rho, x, case.h)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-13 * op_scale(rho, x, case.h))


def check_solution(rho, b, h, p, tol, p_ref=None, linf=1e-7):
    rr = cref.relative_residual(rho, b, p, h)
    assert rr <= tol, f"oracle residual {rr:.3e} > {tol:.1e}"
    assert abs(p.mean()) <= 1e-12 * np.abs(p).max()
    if p_ref is not None:
        err = P.relative_linf_error(p, p_ref)
        assert err < linf, f"L-inf error {err:.3e}"
        return rr, err
    return rr, None


SMALL = [(8, 4, 4), (2, 2, 2), (4, 2, 2), (12, 10, 6), (8, 6, 5), (10, 7, 9), (32, 16, 16), (64, 32, 32)]


@pytest.mark.parametrize("shape", SMALL)
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_solve_small_against_dense_or_reference(shape, mode):
    """Tiny and ragged grids (odd sizes: no coarsening; sizes that stop coarsening
    early: the sweep-based coarsest solve), 833:1 jumps from random gas fractions."""
    nz, ny, nx = shape
    say("solve small", shape, mode)
    case = W.random_small_case(11 + sum(shape), nx, ny, nz)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    n = nx * ny * nz
    p_ref = P.solve_dense(rho_ref, b_ref, case.h) if n <= 1024 else cref.solve(rho_ref, b_ref, case.h, tol=1e-13)[0]
    with ppsolve.Solver(nx, ny, nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
    p = cpu(p)
    rr, err = check_solution(rho_ref, b_ref, case.h, p, 1e-10, p_ref)
    say("   iters", st["iters"], st["inner_iters_total"], "res", rr, "err", err)


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_duct32_against_reference(mode):
    case = W.preset("duct32")
    say("duct32", mode)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    p_ref, it, rr_ref, _ = cref.solve(rho_ref, b_ref, case.h, tol=1e-13)
    assert rr_ref < 1e-13
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
        p = cpu(p)
        rr, err = check_solution(rho_ref, b_ref, case.h, p, 1e-10, p_ref)
        say("   iters", st["iters"], st["inner_iters_total"], "res", rr, "err", err, "ms", st["solve_ms"])
        # bitwise repeatable
        p2, st2 = S.solve(b_t)
        np.testing.assert_array_equal(cpu(p2), p)
        # warm start from the solution: converges immediately
        p3, st3 = S.solve(b_t, gpu(p))
        assert st3["iters"] == 0
        # a constant added to the guess does not change the answer
        p4, _ = S.solve(b_t, gpu(p + 5.0))
        assert P.relative_linf_error(cpu(p4), p_ref) < 1e-7 and abs(cpu(p4).mean()) < 1e-12


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("env", [{"PP_TAILMAX": "8192"}, {"PP_TAIL": "0"}, {"PP_FUSE": "0"}, {"PP_FUSE": "2"},
                                 {"PP_PFUSE": "0"}, {"PP_HW": "0"}],
                         ids=["tail_from_8192", "no_tail", "unfused", "fused_everywhere", "fused_pre_only",
                              "float32_coarse_weights"])
def test_duct32_cycle_variants(mode, env, monkeypatch):
    """The other paths, read from the environment when the handle is made: a
    one-launch tail from the 8192-cell level (its first level read from global
    memory), no tail (a launch per pass, dense product on its own), and the
    passes of a once-smoothed level (first sweep + restriction, prolongation +
    last half-sweep) as separate launches everywhere, fused in float64 as well,
    or fused before the coarse correction only, and float32 (instead of bfloat16)
    face weights on the float32 cycle's large coarse levels."""
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    case = W.preset("duct32")
    say("duct32", mode, env)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    p_ref, it, rr_ref, _ = cref.solve(rho_ref, b_ref, case.h, tol=1e-13)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
        p = cpu(p)
    rr, err = check_solution(rho_ref, b_ref, case.h, p, 1e-10, p_ref)
    say("   iters", st["iters"], st["inner_iters_total"], "res", rr, "err", err, "ms", st["solve_ms"])


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("shape", [(64, 32, 32), (64, 22, 16), (16, 10, 6)])  # (nz, ny, nx)
def test_one_pass_setup_equals_separate_passes(mode, shape, monkeypatch):
    """The set-up's single pass over the density (the handle's density copies,
    the finest 1/D and the first coarse level's face weights, and the density's
    validation) forms every value as the separate passes do: the same solve, bit
    for bit, with either (PP_ONEPASS=0 selects the separate passes)."""
    nz, ny, nx = shape
    case = W.random_small_case(11, nx, ny, nz)
    say("one-pass set-up", mode, shape)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("PP_ONEPASS", flag)
        with ppsolve.Solver(nx, ny, nz, case.h, mode=mode, tol=1e-10) as S:
            S.set_density(rho_t)
            p, st = S.solve(b_t)
            out.append((cpu(p), st["iters"], st["rel_residual"]))
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]
    assert np.array_equal(out[0][0], out[1][0])
    check_solution(rho_ref, b_ref, case.h, out[0][0], 1e-10)


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_back_to_back_set_ups_then_solve(mode):
    """The coarsest level's dense inverse is formed on a second stream and the
    next solve waits for it.  Two set-ups in a row (the second while the first
    one's inverse may still run) and then a solve give, bit for bit, the solve
    of a handle that only saw the second density; a solve right after a set-up
    on a handle that has solved before does too."""
    case = W.preset("duct32")
    other = W.random_small_case(3, case.nx, case.ny, case.nz)
    say("back-to-back set-ups", mode)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    rho_o = ppsolve.density_from_fraction(gpu(other.alpha))
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p_fresh, st_fresh = S.solve(b_t)
        p_fresh = cpu(p_fresh)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_o)
        S.set_density(rho_t)
        p_two, st_two = S.solve(b_t)
        p_two = cpu(p_two)
        S.set_density(rho_o)
        S.solve(b_t)
        S.set_density(rho_t)
        p_again, _ = S.solve(b_t)
        p_again = cpu(p_again)
    assert st_two["iters"] == st_fresh["iters"]
    assert np.array_equal(p_two, p_fresh) and np.array_equal(p_again, p_fresh)
    check_solution(rho_ref, b_ref, case.h, p_fresh, 1e-10)


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
@pytest.mark.parametrize("name", ["duct32", "bubble48"])
def test_tight_tolerance_near_the_rounding_floor(mode, name):
    """Close to the rounding floor the finest-level step length stays accurate:
    its numerator <z, r> - mean(z) sum(r) is <d, r> without the term that the
    previous step's length makes zero, and keeps the mean term, which is not
    small against <z, r> once r is near rounding level.  The solve reaches 1e-13
    on the duct and 1e-12 on the static bubble (whose float64 floor is about
    4.5e-13 with either numerator) instead of stalling at max_iters, and the
    oracle's operator agrees on the residual."""
    if name == "duct32":
        case = W.preset("duct32")
        rho_ref, b_ref, rho_t, b_t = inputs(case)
        nx, ny, nz, h = case.nx, case.ny, case.nz, case.h
    else:
        nx, ny, nz = 48, 48, 64
        h = 1.0 / nx
        a = W.volume_fraction(nx, ny, nz, np.array([[24.3, 23.6, 31.1]]), 19.0)
        rho_ref = P.density_from_fraction(a)
        b_ref = P.surface_tension_rhs(rho_ref, a, 2.0 / (9.5 * h), 0.072, h)
        rho_t, b_t = gpu(rho_ref), gpu(b_ref)
    tol = 1e-13 if name == "duct32" else 1e-12
    say("tight tolerance", name, mode, tol)
    with ppsolve.Solver(nx, ny, nz, h, mode=mode, tol=tol, max_iters=300) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
    p = cpu(p)
    rr = cref.relative_residual(rho_ref, b_ref, p, h)
    say("   iters", st["iters"], "res", st["rel_residual"], "oracle res", rr)
    assert st["rel_residual"] <= tol and st["iters"] < 100
    assert rr <= 2 * tol


@pytest.mark.parametrize("scale", [1e-6, 1e6])
def test_density_scale_far_from_one_refined(scale, monkeypatch):
    """Density times s: every face coefficient is divided by s, so the pressure is
    multiplied by s (the right-hand side is unchanged).  With the float32 cycle's
    coarse weights in bfloat16 on every coarse level (PP_HWMIN=0; by default only
    levels above 65536 cells), weights 1e6 times larger or smaller than usual stay
    finite and non-zero, and the solve still matches the oracle's reference
    pressure."""
    monkeypatch.setenv("PP_HWMIN", "0")
    case = W.preset("duct32")
    say("duct32 density scale", scale)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    p_ref, *_ = cref.solve(rho_ref, b_ref, case.h, tol=1e-13)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode="fp32_refined", tol=1e-10) as S:
        S.set_density(rho_t * scale)
        p, st = S.solve(b_t)
    p = cpu(p)
    rr, err = check_solution(rho_ref * scale, b_ref, case.h, p, 1e-10, p_ref * scale)
    say("   iters", st["iters"], "res", rr, "err", err)


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_duct128_against_reference(mode):
    case = W.preset("duct128")
    say("duct128", mode)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    p_ref, it, rr_ref, secs = cref.solve(rho_ref, b_ref, case.h, tol=1e-13)
    say("   oracle", it, rr_ref, f"{secs:.1f}s")
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
    p = cpu(p)
    rr, err = check_solution(rho_ref, b_ref, case.h, p, 1e-10, p_ref)
    say("   iters", st["iters"], st["inner_iters_total"], "res", rr, "err", err, "ms", st["solve_ms"])


@pytest.fixture(scope="module")
def duct256_reference():
    """256x256x512 with 864 bubbles: the oracle's own inputs and its reference
    pressure, solved to a relative residual of 1e-13 (float64 stagnation sets in
    just below that at this size; the oracle restarts from its true residual until
    the tolerance is met or the iteration cap ends it)."""
    case = W.preset("duct256")
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h)
    p_ref, it, rr, secs = cref.solve(rho, b, case.h, tol=1e-13, maxit=1500)
    say(f"duct256 oracle reference: {it} iterations, residual {rr:.2e}, {secs:.1f} s on {cref.num_threads()} threads")
    assert rr < 2e-13
    return case, rho, b, p_ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_duct256_against_reference(mode, duct256_reference):
    """The headline configuration: 256x256x512, 864 bubbles of 13 cells, 1000:1.2,
    from a zero guess to 1e-10.  Accepted by the oracle's residual, and the pressure
    compared element by element with the oracle's reference pressure (L-inf < 1e-7)."""
    case, rho_ref, b_ref, p_ref = duct256_reference
    say("duct256", mode)
    rho_t = ppsolve.density_from_fraction(gpu(case.alpha))
    b_t = ppsolve.divergence(gpu(case.u), gpu(case.v), gpu(case.w), case.h)
    np.testing.assert_array_equal(cpu(rho_t), rho_ref)
    np.testing.assert_array_equal(cpu(b_t), b_ref)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t)
    p = cpu(p)
    rr, err = check_solution(rho_ref, b_ref, case.h, p, 1e-10, p_ref)
    say("   iters", st["iters"], st["inner_iters_total"], "res", rr, "L-inf err", err, "ms", st["solve_ms"],
        "setup", st["setup_ms"])


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_duct256_uniform_density_against_spectral(mode):
    """Uniform density at 256x256x512: A = L / rho0 is diagonalised by the cosine
    transform in x, y and the Fourier transform in z, so the spectral solve is exact
    to rounding at any size.  The GPU solve from a zero guess must match it."""
    case = W.preset("duct256")
    rho0 = 1000.0
    b = P.divergence(case.u, case.v, case.w, case.h)
    p_ref = P.solve_spectral(rho0, b, case.h)
    say("duct256 uniform density", mode)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, mode=mode, tol=1e-10) as S:
        S.set_density(torch.full(b.shape, rho0, dtype=torch.float64, device=DEV))
        p, st = S.solve(gpu(b))
    p = cpu(p)
    rr, err = check_solution(np.full(b.shape, rho0), b, case.h, p, 1e-10, p_ref)
    say("   iters", st["iters"], "res", rr, "L-inf err", err)


def test_errors_and_degenerate_inputs():
    say("errors")
    nx, ny, nz = 8, 8, 16
    case = W.random_small_case(5, nx, ny, nz)
    rho_ref, b_ref, rho_t, b_t = inputs(case)
    with ppsolve.Solver(nx, ny, nz) as S:
        with pytest.raises(ppsolve.PPError) as e:
            S.solve(b_t)
        assert e.value.code == ppsolve.PP_ERR_STATE
        bad = rho_t.clone()
        bad[3, 2, 1] = float("nan")
        with pytest.raises(ppsolve.PPError) as e:
            S.set_density(bad)
        assert e.value.code == ppsolve.PP_ERR_NONFINITE
        bad = rho_t.clone()
        bad[0, 0, 0] = -1.0
        with pytest.raises(ppsolve.PPError) as e:
            S.set_density(bad)
        assert e.value.code == ppsolve.PP_ERR_NONFINITE
        S.set_density(rho_t)
        # zero and constant right-hand sides: the answer is p = 0
        for rhs in (torch.zeros_like(b_t), torch.full_like(b_t, 3.0)):
            p, st = S.solve(rhs, torch.ones_like(b_t))
            assert torch.count_nonzero(p).item() == 0 and st["iters"] == 0
        bb = b_t.clone()
        bb[1, 1, 1] = float("inf")
        with pytest.raises(ppsolve.PPError) as e:
            S.solve(bb)
        assert e.value.code == ppsolve.PP_ERR_NONFINITE
    with ppsolve.Solver(nx, ny, nz, max_iters=1, tol=1e-14) as S:
        S.set_density(rho_t)
        p, st = S.solve(b_t, check=False)
        assert st["status"] == ppsolve.PP_ERR_NOT_CONVERGED
        assert st["iters"] == 1 and 0 < st["rel_residual"] < 1
        assert torch.isfinite(p).all()
