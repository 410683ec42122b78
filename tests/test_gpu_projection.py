"""Steps around the solve on the GPU: face projection and the surface-tension pressure.

* projection (step 12 on faces): bit-exact against the oracle for the same
  pressure; after a solve of step 11 the projected velocity's divergence is
  dt times the solve's residual.
* surface tension (eq. ppe_surface_tension with eq. jump_condition as source):
  the right-hand side is bit-exact against the oracle; for a static bubble with
  exact (constant) curvature the solved pressure is sigma*kappa*(a - mean a) and
  the face velocity it leaves is zero to rounding.
"""
import numpy as np
import pytest
import torch

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def c(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name", ["duct32", "duct128"])
def test_projection_removes_divergence(name):
    print("projection", name, flush=True)
    case = W.preset(name)
    dt = 0.5
    rho_t = ppsolve.density_from_fraction(g(case.alpha))
    u_t, v_t, w_t = g(case.u), g(case.v), g(case.w)
    b_t = ppsolve.divergence(u_t, v_t, w_t, case.h, dt)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=1e-12) as S:
        S.set_density(rho_t)
        p_t, st = S.solve(b_t)
    p = c(p_t)
    rho = P.density_from_fraction(case.alpha)
    un, vn, wn = P.project(rho, p, case.u, case.v, case.w, case.h, dt)
    ppsolve.project(rho_t, p_t, u_t, v_t, w_t, case.h, dt)
    np.testing.assert_array_equal(c(u_t), un)
    np.testing.assert_array_equal(c(v_t), vn)
    np.testing.assert_array_equal(c(w_t), wn)
    d_new = c(ppsolve.divergence(u_t, v_t, w_t, case.h))
    b = P.divergence(case.u, case.v, case.w, case.h, dt)
    assert np.max(np.abs(d_new - d_new.mean())) < 1e-9 * np.max(np.abs(b))
    print("   max |div u_new| / max |div u| =", np.max(np.abs(d_new)) / np.max(np.abs(b)), flush=True)


@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_static_bubble_surface_tension_balance(mode):
    print("static bubble", mode, flush=True)
    nx, ny, nz = 48, 48, 64
    h = 1.0 / nx
    R = 9.5
    a = W.volume_fraction(nx, ny, nz, np.array([[24.3, 23.6, 31.1]]), 2 * R)
    rho = P.density_from_fraction(a)
    sigma, kappa = 0.072, 2.0 / (R * h)
    kap = np.full(a.shape, kappa)
    rhs_ref = P.surface_tension_rhs(rho, a, kappa, sigma, h)
    rho_t, a_t, k_t = g(rho), g(a), g(kap)
    rhs_t = ppsolve.surface_tension_rhs(rho_t, a_t, k_t, sigma, h)
    np.testing.assert_array_equal(c(rhs_t), rhs_ref)
    with ppsolve.Solver(nx, ny, nz, h, mode=mode, tol=1e-11) as S:
        S.set_density(rho_t)
        p_t, st = S.solve(rhs_t)
    p = c(p_t)
    exact = sigma * kappa * (a - a.mean())
    err = P.relative_linf_error(p, exact)
    bx, by, bz = P.face_coefficients(rho)
    fx, fy, fz = P.surface_force(a, kappa, sigma, h)
    gx, gy, gz = P.gradient(p, h)
    spurious = max(np.max(np.abs(bx * (fx - gx))), np.max(np.abs(by * (fy - gy))), np.max(np.abs(bz * (fz - gz))))
    scale = np.max(np.abs(bz * fz))
    print(f"   pressure jump error {err:.2e}; spurious face velocity / force scale {spurious / scale:.2e}", flush=True)
    assert err < 1e-8
    assert spurious < 1e-8 * scale
    assert cref.relative_residual(rho, rhs_ref, p, h) <= 1e-11


@pytest.mark.parametrize("shape", [(101, 256, 256), (7, 33, 5), (512, 256, 256)])
def test_projection_and_surface_rhs_bitexact_multi_plane(shape):
    """The divergence, projection and surface-tension kernels walk a z range per
    thread, carry values from plane to plane and share neighbour values between
    lanes and rows of a tile.  At 256 x 256 x 101 a thread walks 4 planes and the last z
    range holds 1; 5 x 33 x 7 is a ragged cross-section; 256 x 256 x 512 is the
    benchmark's size and launch (16 planes per thread).  Random fields, so no
    face value is special; all three must match the oracle bit for bit."""
    nz, ny, nx = shape
    print("multi-plane", shape, flush=True)
    rng = np.random.default_rng(11)
    h = 1.0 / nx
    a = rng.random(shape)
    rho = P.density_from_fraction(a)
    kap = rng.normal(size=shape) * 40.0
    p = rng.normal(size=shape)
    u, v, w = (rng.normal(size=shape) for _ in range(3))
    rhs_ref = P.surface_tension_rhs(rho, a, kap, 0.072, h)
    np.testing.assert_array_equal(c(ppsolve.surface_tension_rhs(g(rho), g(a), g(kap), 0.072, h)), rhs_ref)
    np.testing.assert_array_equal(c(ppsolve.divergence(g(u), g(v), g(w), h, 0.5)), P.divergence(u, v, w, h, 0.5))
    un, vn, wn = P.project(rho, p, u, v, w, h, 0.25)
    u_t, v_t, w_t = g(u), g(v), g(w)
    ppsolve.project(g(rho), g(p), u_t, v_t, w_t, h, 0.25)
    np.testing.assert_array_equal(c(u_t), un)
    np.testing.assert_array_equal(c(v_t), vn)
    np.testing.assert_array_equal(c(w_t), wn)


SHAPES = [(2, 2, 2), (3, 5, 4), (7, 6, 8), (16, 8, 8), (33, 17, 10), (64, 32, 32), (512, 256, 256)]  # (nz, ny, nx)


@pytest.mark.parametrize("with_pt", [False, True], ids=["p_only", "p_and_pt"])
@pytest.mark.parametrize("shape", SHAPES)
def test_correct_velocity_bit_exact(shape, with_pt):
    """Step 12 on faces and cells in one pass (pp_correct_velocity) against the
    oracle's face projection and cell correction, bit for bit, with and without
    the surface-tension pressure; ragged tiles and the full 256x256x512 grid."""
    nz, ny, nx = shape
    print("correct_velocity", shape, with_pt, flush=True)
    case = W.preset("duct256") if nx == 256 else W.random_small_case(70 + sum(shape), nx, ny, nz)
    rng = np.random.default_rng(sum(shape))
    rho = P.density_from_fraction(case.alpha)
    p = rng.standard_normal(shape)
    pt = rng.standard_normal(shape) * 0.1 if with_pt else None
    uc, vc, wc = (rng.standard_normal(shape) for _ in range(3))
    dt = 0.37
    un, vn, wn = P.project(rho, p, case.u, case.v, case.w, case.h, dt)
    ucn, vcn, wcn = P.correct_cell_velocity(rho, p, pt, uc, vc, wc, case.h, dt)
    ts = [g(a) for a in (case.u, case.v, case.w, uc, vc, wc)]
    ppsolve.correct_velocity(g(rho), g(p), g(pt) if with_pt else None, *ts, case.h, dt)
    for got, want in zip(ts, (un, vn, wn, ucn, vcn, wcn)):
        np.testing.assert_array_equal(c(got), want)


def test_correct_velocity_after_solve_removes_divergence_and_matches_average():
    """After the step-11 solve the corrected face velocities are divergence-free to
    the solve's residual, and the cell correction equals the face correction
    averaged to the cells."""
    case = W.preset("duct32")
    dt = 0.5
    rho_t = ppsolve.density_from_fraction(g(case.alpha))
    u_t, v_t, w_t = g(case.u), g(case.v), g(case.w)
    b_t = ppsolve.divergence(u_t, v_t, w_t, case.h, dt)
    with ppsolve.Solver(case.nx, case.ny, case.nz, case.h, tol=1e-12) as S:
        S.set_density(rho_t)
        p_t, _ = S.solve(b_t)
    zero = [torch.zeros_like(u_t) for _ in range(3)]
    ppsolve.correct_velocity(rho_t, p_t, None, u_t, v_t, w_t, *zero, case.h, dt)
    d_new = c(ppsolve.divergence(u_t, v_t, w_t, case.h))
    b = P.divergence(case.u, case.v, case.w, case.h, dt)
    assert np.max(np.abs(d_new - d_new.mean())) < 1e-9 * np.max(np.abs(b))
    du, dv, dw = case.u - c(u_t), case.v - c(v_t), case.w - c(w_t)
    du[:, :, -1] = 0.0
    dv[:, -1, :] = 0.0
    ax, ay, az = P.face_to_cell(du, dv, dw)
    for got, want in zip(zero, (ax, ay, az)):
        np.testing.assert_allclose(-c(got), want, rtol=0, atol=1e-12 * np.abs(want).max())
