"""Pins of the CPU oracle against facts other than itself (no GPU needed).

Each test ties one oracle function to something it does not compute itself:
an independent sparse construction, a library routine, a closed form, an
invariant of the mathematics, brute force, or a value printed in the paper.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.stats

from oracle import cref, poisson as P, relax as R
from paper_2104_01636_amd import workload as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_rho(shape, seed):
    """Density with the 833:1 jumps: gas fraction drawn from {0, 1/64, ..., 1}."""
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 65, size=shape) / 64.0
    return 1000.0 * (1.0 - a) + 1.2 * a


# ------------------------------------------------------------------ sparse construction (test side)

def incidence(nx, ny, nz):
    """Face-by-cell incidence G (rows: interior x faces, interior y faces, all z
    faces; +1 on the far cell, -1 on the near cell) and the matching face
    index into the (nz, ny, nx) face arrays."""
    rows, cols, vals, fidx = [], [], [], []
    r = 0

    def cid(i, j, k):
        return i + nx * (j + ny * k)

    for axis in range(3):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    if axis == 0:
                        if i == nx - 1:
                            continue
                        a, b = cid(i, j, k), cid(i + 1, j, k)
                    elif axis == 1:
                        if j == ny - 1:
                            continue
                        a, b = cid(i, j, k), cid(i, j + 1, k)
                    else:
                        a, b = cid(i, j, k), cid(i, j, (k + 1) % nz)
                    rows += [r, r]
                    cols += [b, a]
                    vals += [1.0, -1.0]
                    fidx.append((axis, cid(i, j, k)))
                    r += 1
    G = sp.csr_matrix((vals, (rows, cols)), shape=(r, nx * ny * nz))
    return G, fidx


def face_vector(fidx, faces):
    return np.array([faces[a].ravel()[c] for a, c in fidx])


def sparse_operator(rho, h):
    """A = -G^T diag(beta) G / h^2, with beta = 1/mean(rho_L, rho_R) from scipy.stats.hmean."""
    nz, ny, nx = rho.shape
    G, fidx = incidence(nx, ny, nz)
    r = rho.ravel()
    beta = []
    for row in range(G.shape[0]):
        cells = G.indices[G.indptr[row]:G.indptr[row + 1]]
        beta.append(scipy.stats.hmean([1.0 / r[cells[0]], 1.0 / r[cells[1]]]))
    return -(G.T @ sp.diags(np.array(beta)) @ G) / h ** 2


# ------------------------------------------------------------------ density, coefficients

def test_density_from_fraction_endpoints_and_paper_ratio():
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    a = np.array([0.0, 1.0, 0.5, 0.25])
    rho = P.density_from_fraction(a)
    assert rho[0] == g["rho_liquid"] and rho[1] == g["rho_gas"]
    assert rho[2] == pytest.approx(0.5 * (1000.0 + 1.2), rel=1e-15)
    assert round(rho[0] / rho[1]) == g["density_ratio_printed"]
    np.testing.assert_array_equal(cref.density_from_fraction(a), rho)


def test_face_coefficient_is_harmonic_mean_of_inverse_density():
    rho = rand_rho((4, 3, 5), 7)
    bx, by, bz = P.face_coefficients(rho)
    nz, ny, nx = rho.shape
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                if i < nx - 1:
                    assert bx[k, j, i] == pytest.approx(scipy.stats.hmean([1 / rho[k, j, i], 1 / rho[k, j, i + 1]]), rel=1e-15)
                else:
                    assert bx[k, j, i] == 0.0
                if j < ny - 1:
                    assert by[k, j, i] == pytest.approx(scipy.stats.hmean([1 / rho[k, j, i], 1 / rho[k, j + 1, i]]), rel=1e-15)
                else:
                    assert by[k, j, i] == 0.0
                kp = (k + 1) % nz
                assert bz[k, j, i] == pytest.approx(scipy.stats.hmean([1 / rho[k, j, i], 1 / rho[kp, j, i]]), rel=1e-15)
    # uniform density: every interior face coefficient is exactly 1/rho
    bxu, byu, bzu = P.face_coefficients(np.full((2, 2, 2), 4.0))
    assert np.all(bzu == 0.25) and np.all(bxu[:, :, 0] == 0.25)
    for a, b in zip(cref.face_coefficients(rho), (bx, by, bz)):
        np.testing.assert_array_equal(a, b)


# ------------------------------------------------------------------ operator

@pytest.mark.parametrize("shape", [(4, 3, 5), (2, 2, 2), (6, 4, 4), (2, 5, 3), (8, 2, 2)])
def test_operator_matches_sparse_incidence_construction(shape):
    h = 1.0 / shape[2]
    rho = rand_rho(shape, sum(shape))
    p = np.random.default_rng(3).standard_normal(shape)
    A = sparse_operator(rho, h)
    ref = (A @ p.ravel()).reshape(shape)
    scale = np.max(np.abs(ref))
    np.testing.assert_allclose(P.apply_operator(rho, p, h), ref, rtol=0, atol=1e-13 * scale)
    np.testing.assert_allclose(cref.apply_operator(rho, p, h), ref, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("shape", [(4, 3, 5), (6, 4, 4), (2, 5, 3)])
def test_relative_residual_two_sided_against_sparse_operator(shape):
    """The acceptance number ||bbar - A p|| / ||bbar|| (bbar = b - mean b) of both
    oracle implementations equals the one formed from the sparse incidence operator,
    on iterates far from converged (so a ratio that is squared, not mean-shifted, or
    normalised by ||b|| instead of ||bbar||, differs by far more than the tolerance)."""
    h = 1.0 / shape[2]
    rho = rand_rho(shape, 40 + sum(shape))
    rng = np.random.default_rng(41)
    b = rng.standard_normal(shape) + 3.0          # mean far from zero: bbar != b
    A = sparse_operator(rho, h)
    bb = b.ravel() - b.mean()
    p_exact = P.solve_dense(rho, b, h)
    for mix in (0.0, 0.5, 0.9, 1.0 - 1e-6):
        p = mix * p_exact + (1.0 - mix) * rng.standard_normal(shape) * np.abs(p_exact).max()
        expect = np.linalg.norm(bb - A @ p.ravel()) / np.linalg.norm(bb)
        assert 1e-7 < expect
        got_py = P.relative_residual(rho, b, p, h)
        got_c = cref.relative_residual(rho, b, p, h)
        assert got_py == pytest.approx(expect, rel=1e-12)
        assert got_c == pytest.approx(expect, rel=1e-12)
    # the exact solution: residual at the rounding level, and a constant shift changes nothing
    assert P.relative_residual(rho, b, p_exact + 11.0, h) < 1e-12
    assert cref.relative_residual(rho, b, p_exact + 11.0, h) < 1e-12


def test_relative_linf_error_worked_values():
    """||(p - mean p) - (q - mean q)||_inf / ||q - mean q||_inf on hand-computed cases."""
    q = np.array([1.0, -1.0, 2.0, -2.0])                       # zero mean, max |q| = 2
    assert P.relative_linf_error(q + np.array([0.1, 0.0, 0.0, -0.1]) + 7.0, q) == pytest.approx(0.05, rel=1e-14)
    # a perturbation with mean 0.1: after removing it the difference is (0.3, -0.1, -0.1, -0.1)
    assert P.relative_linf_error(q + np.array([0.4, 0.0, 0.0, 0.0]), q) == pytest.approx(0.15, rel=1e-14)
    # the reference's own mean is removed before its norm is taken: q + 5 has the same error
    assert P.relative_linf_error(q + np.array([0.4, 0.0, 0.0, 0.0]), q + 5.0) == pytest.approx(0.15, rel=1e-14)
    assert P.relative_linf_error(-q, q) == pytest.approx(2.0, rel=1e-15)


def test_operator_invariants_and_null_space():
    shape = (8, 4, 4)
    h = 0.25
    rho = rand_rho(shape, 11)
    A = P.assemble_dense(rho, h)
    scale = np.max(np.abs(A))
    np.testing.assert_allclose(A, A.T, rtol=0, atol=1e-14 * scale)          # symmetric
    np.testing.assert_allclose(A @ np.ones(A.shape[0]), 0.0, atol=1e-13 * scale)   # A 1 = 0
    np.testing.assert_allclose(np.ones(A.shape[0]) @ A, 0.0, atol=1e-13 * scale)   # 1^T A = 0
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-10 * scale                     # negative semi-definite
    assert np.sum(np.abs(ev) < 1e-9 * scale) == 1       # kernel = constants only
    u = np.random.default_rng(1).standard_normal(A.shape[0])
    u -= u.mean()
    assert u @ A @ u < 0.0


def test_operator_eigenmodes_closed_form():
    """Uniform density: cos(pi l (i+1/2)/nx) cos(pi m (j+1/2)/ny) exp(2 pi i n k/nz)
    are eigenvectors with eigenvalue -(4/h^2)[sin^2(pi l/2nx) + sin^2(pi m/2ny) + sin^2(pi n/nz)]/rho."""
    nz, ny, nx, h, rho0 = 12, 6, 10, 0.1, 3.0
    i = np.arange(nx); j = np.arange(ny); k = np.arange(nz)
    for (l, m, n) in [(1, 0, 0), (3, 2, 1), (0, 5, 6), (9, 1, 11)]:
        mode = (np.cos(np.pi * n * 0 + 2 * np.pi * n * k / nz)[:, None, None]
                * np.cos(np.pi * m * (j + 0.5) / ny)[None, :, None]
                * np.cos(np.pi * l * (i + 0.5) / nx)[None, None, :])
        lam = -(4.0 / h ** 2) * (np.sin(np.pi * l / (2 * nx)) ** 2 + np.sin(np.pi * m / (2 * ny)) ** 2
                                 + np.sin(np.pi * n / nz) ** 2) / rho0
        got = P.apply_operator(np.full((nz, ny, nx), rho0), mode, h)
        np.testing.assert_allclose(got, lam * mode, rtol=0, atol=1e-11 * abs(lam))


# ------------------------------------------------------------------ divergence

def test_divergence_gauss_and_summation_by_parts():
    case = W.random_small_case(5, 6, 5, 8)
    h = case.h
    d = P.divergence(case.u, case.v, case.w, h)
    assert abs(d.sum()) < 1e-12 * np.abs(d).max() * d.size      # net outflow through the walls is zero
    p = np.random.default_rng(2).standard_normal(d.shape)
    gx, gy, gz = P.gradient(p, h)
    # <div u, p> = -<u, grad p> over faces (walls carry no flux)
    lhs = np.sum(d * p)
    rhs = -(np.sum(case.u * gx) + np.sum(case.v * gy) + np.sum(case.w * gz))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    np.testing.assert_array_equal(cref.divergence(case.u, case.v, case.w, h), d)


def test_divergence_linear_field_closed_form():
    nz, ny, nx, h = 4, 3, 6, 0.5
    xf = (np.arange(nx) + 1.0) * h          # position of the +x face of each cell
    u = np.broadcast_to(xf, (nz, ny, nx)).copy()
    zero = np.zeros((nz, ny, nx))
    d = P.divergence(u, zero, zero, h, dt=2.0)
    expect = np.full((nz, ny, nx), 0.5)      # (h / h) / dt
    expect[:, :, -1] = -(nx - 1) * h / h / 2.0  # the east wall carries zero
    np.testing.assert_allclose(d, expect, rtol=1e-15)


# ------------------------------------------------------------------ solves

@pytest.mark.parametrize("shape", [(8, 4, 4), (4, 2, 2), (8, 3, 5)])
def test_spectral_matches_dense_uniform_density(shape):
    h = 1.0 / shape[2]
    b = np.random.default_rng(4).standard_normal(shape)
    rho0 = 7.0
    ps = P.solve_spectral(rho0, b, h)
    pd = P.solve_dense(np.full(shape, rho0), b, h)
    assert P.relative_linf_error(ps, pd) < 1e-12
    assert P.relative_residual(np.full(shape, rho0), b, ps, h) < 1e-12


@pytest.mark.parametrize("shape", [(8, 4, 4), (16, 8, 8), (2, 2, 2), (6, 4, 2)])
def test_c_solver_matches_dense_with_density_jumps(shape):
    h = 1.0 / shape[2]
    rho = rand_rho(shape, 21)
    b = np.random.default_rng(5).standard_normal(shape)
    pd = P.solve_dense(rho, b, h)
    assert P.relative_residual(rho, b, pd, h) < 1e-11
    pc, it, rr, _ = cref.solve(rho, b, h, tol=1e-14, maxit=400)
    assert rr < 1e-12
    assert P.relative_linf_error(pc, pd) < 1e-10
    assert abs(pc.mean()) < 1e-14 * np.abs(pc).max()


def test_c_solver_matches_spectral_uniform_density():
    shape = (64, 32, 32)
    h = 1.0 / 32
    b = np.random.default_rng(6).standard_normal(shape)
    ps = P.solve_spectral(1000.0, b, h)
    pc, it, rr, _ = cref.solve(np.full(shape, 1000.0), b, h, tol=1e-13)
    assert rr < 1e-13
    assert P.relative_linf_error(pc, ps) < 1e-11


def test_manufactured_solution_second_order():
    errs = []
    for n in (16, 32, 64):
        h = 1.0 / n
        rho, f, p_exact = P.manufactured(n, n, 2 * n, h)
        p, it, rr, _ = cref.solve(rho, f, h, tol=1e-12)
        assert rr < 1e-12
        errs.append(np.max(np.abs(p - p_exact)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(orders > 1.85) and np.all(orders < 2.15), (errs, orders)


def test_metamorphic_relations():
    case = W.make_case(16, 16, 32, 4, 6.0, seed=9)
    h = case.h
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, h)
    p, *_ = cref.solve(rho, b, h, tol=1e-13)
    tol = 1e-9
    # density scaling: A -> A/c, so p -> c p
    p2, *_ = cref.solve(3.0 * rho, b, h, tol=1e-13)
    assert P.relative_linf_error(p2, 3.0 * p) < tol
    # right-hand-side scaling
    p3, *_ = cref.solve(rho, -2.5 * b, h, tol=1e-13)
    assert P.relative_linf_error(p3, -2.5 * p) < tol
    # periodic roll in z
    p4, *_ = cref.solve(np.roll(rho, 5, axis=0), np.roll(b, 5, axis=0), h, tol=1e-13)
    assert P.relative_linf_error(p4, np.roll(p, 5, axis=0)) < tol
    # mirror in x
    p5, *_ = cref.solve(rho[:, :, ::-1], b[:, :, ::-1], h, tol=1e-13)
    assert P.relative_linf_error(p5, p[:, :, ::-1]) < tol
    # transpose x <-> y
    p6, *_ = cref.solve(rho.transpose(0, 2, 1), b.transpose(0, 2, 1), h, tol=1e-13)
    assert P.relative_linf_error(p6, p.transpose(0, 2, 1)) < tol


def test_residual_is_divergence_of_projected_velocity():
    """D(u - dt beta G p) = dt (b - A p) with b = D u / dt: the solve's residual
    is the divergence left in the corrected velocity (step 12's convention)."""
    case = W.random_small_case(8, 6, 4, 8)
    h, dt = case.h, 0.3
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, h, dt)
    p = P.solve_dense(rho, b, h)
    bx, by, bz = P.face_coefficients(rho)
    gx, gy, gz = P.gradient(p, h)
    un = case.u - dt * bx * gx
    vn = case.v - dt * by * gy
    wn = case.w - dt * bz * gz
    d_new = P.divergence(un, vn, wn, h)
    np.testing.assert_allclose(d_new, dt * (b - P.apply_operator(rho, p, h)), atol=1e-9)
    assert np.max(np.abs(d_new - dt * b.mean())) < 1e-9 * np.max(np.abs(b))


# ------------------------------------------------------------------ multigrid pieces

def injection_matrix(nx, ny, nz):
    cnx, cny, cnz = nx // 2, ny // 2, nz // 2
    rows = np.arange(nx * ny * nz)
    k, j, i = np.unravel_index(rows, (nz, ny, nx))
    cols = (i // 2) + cnx * ((j // 2) + cny * (k // 2))
    return sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(rows.size, cnx * cny * cnz))


def k_sparse(Wt):
    nz, ny, nx = Wt[0].shape
    G, fidx = incidence(nx, ny, nz)
    w = face_vector(fidx, Wt)
    return G.T @ sp.diags(w) @ G


def test_coarsening_is_galerkin_product():
    shape = (8, 6, 4)
    rho = rand_rho(shape, 3)
    Wf = R.fine_weights(rho)
    Kf = k_sparse(Wf)
    Pm = injection_matrix(shape[2], shape[1], shape[0])
    Kc_ref = (Pm.T @ Kf @ Pm).toarray()
    Kc = k_sparse(R.coarsen_weights(Wf)).toarray()
    np.testing.assert_allclose(Kc, Kc_ref, rtol=0, atol=1e-15 * np.abs(Kc_ref).max())
    r = np.random.default_rng(0).standard_normal(shape)
    np.testing.assert_allclose(R.restrict_sum(r).ravel(), Pm.T @ r.ravel(), atol=1e-14)
    e = np.random.default_rng(1).standard_normal((4, 3, 2))
    np.testing.assert_array_equal(R.prolong_inject(e).ravel(), Pm @ e.ravel())
    # the level operator matches the sparse one and -h^2 A on the finest level
    x = np.random.default_rng(2).standard_normal(shape)
    np.testing.assert_allclose(R.apply_k(Wf, x).ravel(), Kf @ x.ravel(), atol=1e-13)
    h = 0.5
    np.testing.assert_allclose(R.apply_k(Wf, x), -h * h * P.apply_operator(rho, x, h), atol=1e-13)


@pytest.mark.parametrize("colour", [0, 1])
def test_halfsweep_zeroes_residual_on_its_colour(colour):
    shape = (6, 4, 5)
    Wf = R.fine_weights(rand_rho(shape, 4))
    rng = np.random.default_rng(colour)
    x0, f = rng.standard_normal(shape), rng.standard_normal(shape)
    x1 = R.rb_halfsweep(Wf, x0, f, colour, omega=1.0)
    res = f - R.apply_k(Wf, x1)
    m = R.colour_mask(shape, colour)
    assert np.max(np.abs(res[m])) < 1e-12 * np.max(np.abs(f))
    np.testing.assert_array_equal(x1[~m], x0[~m])
    xs = R.rb_halfsweep_sequential(Wf, x0, f, colour, omega=1.0)
    np.testing.assert_allclose(x1, xs, rtol=1e-13, atol=1e-13)
    # SOR: omega blends old and Gauss-Seidel values
    xw = R.rb_halfsweep(Wf, x0, f, colour, omega=1.5)
    np.testing.assert_allclose(xw[m], (-0.5 * x0 + 1.5 * x1)[m], rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ generator

def test_paper_lattice_void_fraction():
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    case = W.paper_lattice_case()
    assert (case.nx, case.ny, case.nz) == tuple(g["grid_cells"])
    assert len(case.centres) == g["n_bubbles"]
    # 2 mm on a 48 mm / 192-cell duct is 8 cells
    assert g["bubble_diameter_mm"] / (g["duct_mm"][0] / g["grid_cells"][0]) == case.diameter
    exact = g["n_bubbles"] * np.pi / 6 * g["bubble_diameter_mm"] ** 3 / np.prod(g["duct_mm"])
    assert round(100 * exact, 2) == g["void_fraction_percent_printed"]
    assert abs(case.alpha.mean() - exact) < 0.01 * exact


@pytest.mark.parametrize("name,void", [("duct32", 0.0327), ("duct128", 0.0552)])
def test_generator_void_fraction_and_spacing(name, void):
    case = W.preset(name)
    a = case.alpha
    assert np.all((a * 64) == np.round(a * 64)) and a.min() == 0.0 and a.max() == 1.0
    exact = len(case.centres) * np.pi / 6 * case.diameter ** 3 / case.n_cells
    assert abs(a.mean() - exact) < 0.005 * exact
    assert round(exact, 4) == void
    c = case.centres
    d = c[:, None, :] - c[None, :, :]
    d[..., 2] -= case.nz * np.round(d[..., 2] / case.nz)
    dist = np.sqrt((d ** 2).sum(-1)) + np.eye(len(c)) * 1e9
    assert dist.min() >= case.diameter
    # same seed, same bits
    again = W.preset(name)
    np.testing.assert_array_equal(again.alpha, a)
    np.testing.assert_array_equal(again.u, case.u)


def test_generator_union_and_wrap():
    # two overlapping bubbles: union, not sum; one bubble across the periodic seam
    a = W.volume_fraction(16, 16, 16, np.array([[8.0, 8.0, 8.0], [9.0, 8.0, 8.0]]), 6.0)
    assert a.max() == 1.0
    b = W.volume_fraction(16, 16, 16, np.array([[8.0, 8.0, 0.5]]), 6.0)
    c = W.volume_fraction(16, 16, 16, np.array([[8.0, 8.0, 8.5]]), 6.0)
    np.testing.assert_array_equal(np.roll(b, 8, axis=0), c)
    # brute force on one bubble: every sub-cell centre tested
    cen = np.array([[5.3, 6.1, 3.7]])
    fast = W.volume_fraction(12, 12, 8, cen, 5.0)
    g = (np.arange(12 * 4) + 0.5) / 4
    gz = (np.arange(8 * 4) + 0.5) / 4
    Z, Y, X = np.meshgrid(gz, g, g, indexing="ij")
    dz = Z - cen[0, 2]
    dz -= 8 * np.round(dz / 8)
    inside = ((X - cen[0, 0]) ** 2 + (Y - cen[0, 1]) ** 2 + dz ** 2) < 2.5 ** 2
    brute = inside.reshape(8, 4, 12, 4, 12, 4).sum(axis=(1, 3, 5)) / 64.0
    np.testing.assert_array_equal(fast, brute)


# ------------------------------------------------------------------ projection and surface tension

def test_projection_leaves_divergence_equal_to_residual():
    case = W.random_small_case(12, 6, 5, 8)
    h, dt = case.h, 0.25
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, h, dt)
    p = P.solve_dense(rho, b, h)
    un, vn, wn = P.project(rho, p, case.u, case.v, case.w, h, dt)
    d = P.divergence(un, vn, wn, h)
    np.testing.assert_allclose(d, dt * (b - b.mean() - P.apply_operator(rho, p, h)) + dt * b.mean(), atol=1e-9)
    assert np.max(np.abs(d - d.mean())) < 1e-9 * np.max(np.abs(b))


def test_static_bubble_exact_curvature_balances_to_machine_zero():
    """Section 2.1: with exact curvature the surface-tension pressure cancels the
    interface force exactly.  For constant kappa the discrete solution is
    p~ = sigma kappa (a - mean a), and the face velocity it drives is zero."""
    nx = 16
    h = 1.0 / nx
    a = W.volume_fraction(nx, nx, 16, np.array([[8.3, 7.6, 8.1]]), 7.0)
    rho = P.density_from_fraction(a)
    sigma, kappa = 0.072, 2.0 / (3.5 * h)
    rhs = P.surface_tension_rhs(rho, a, kappa, sigma, h)
    p = P.solve_dense(rho, rhs, h) if a.size <= 4096 else None
    exact = sigma * kappa * (a - a.mean())
    assert P.relative_linf_error(p, exact) < 1e-9
    bx, by, bz = P.face_coefficients(rho)
    fx, fy, fz = P.surface_force(a, kappa, sigma, h)
    gx, gy, gz = P.gradient(p, h)
    spurious = max(np.max(np.abs(bx * (fx - gx))), np.max(np.abs(by * (fy - gy))), np.max(np.abs(bz * (fz - gz))))
    scale = np.max(np.abs(bx * fx))
    assert spurious < 1e-9 * scale


# ------------------------------------------------------------------ step 12 on cells

def test_face_to_cell_closed_forms():
    """A constant face field averages to itself away from the walls and to half of
    itself in the cells on a wall (the wall face carries zero); a linear face
    field averages to its value at the cell centre."""
    nz, ny, nx = 6, 5, 7
    one = np.ones((nz, ny, nx))
    ax, ay, az = P.face_to_cell(3.0 * one, -2.0 * one, 0.5 * one)
    np.testing.assert_array_equal(az, 0.5 * one)                      # z periodic: no walls
    np.testing.assert_array_equal(ax[:, :, 1:-1], 3.0 * one[:, :, 1:-1])
    np.testing.assert_array_equal(ax[:, :, 0], 1.5 * one[:, :, 0])
    np.testing.assert_array_equal(ax[:, :, -1], 1.5 * one[:, :, -1])
    np.testing.assert_array_equal(ay[:, 1:-1, :], -2.0 * one[:, 1:-1, :])
    np.testing.assert_array_equal(ay[:, 0, :], -1.0 * one[:, 0, :])
    # face value = position of the face (i + 1) along x: the average is the centre i + 1/2
    xf = np.broadcast_to(np.arange(nx) + 1.0, (nz, ny, nx))
    ax, _, _ = P.face_to_cell(xf, 0 * one, 0 * one)
    np.testing.assert_allclose(ax[:, :, 1:-1], (np.arange(nx) + 0.5)[1:-1] * one[:, :, 1:-1], rtol=0, atol=1e-15)


def test_cell_correction_linear_pressure_and_density_scaling():
    """A pressure linear in z with uniform density gives a uniform face gradient
    beta G away from the seam; every cell away from it is corrected by exactly
    dt * G / rho in w and not at all in u, v.  Splitting the pressure between p
    and pt gives the same correction, and a density c times larger gives a
    correction c times smaller."""
    nz, ny, nx, h, dt, rho0 = 8, 4, 5, 0.25, 0.5, 4.0
    z = (np.arange(nz) + 0.5) * h
    p = np.broadcast_to((3.0 * z)[:, None, None], (nz, ny, nx)).copy()
    rho = np.full((nz, ny, nx), rho0)
    uc, vc, wc = (np.random.default_rng(k).standard_normal((nz, ny, nx)) for k in range(3))
    un, vn, wn = P.correct_cell_velocity(rho, p, None, uc, vc, wc, h, dt)
    np.testing.assert_array_equal(un, uc)
    np.testing.assert_array_equal(vn, vc)
    inner = slice(1, nz - 1)   # the faces at the periodic seam see the jump of the linear ramp
    np.testing.assert_allclose(wn[inner], wc[inner] - dt * 3.0 / rho0, rtol=0, atol=1e-14)
    un2, vn2, wn2 = P.correct_cell_velocity(rho, 0.25 * p, 0.75 * p, uc, vc, wc, h, dt)
    np.testing.assert_allclose(wn2, wn, rtol=0, atol=1e-14)
    _, _, wn3 = P.correct_cell_velocity(10.0 * rho, p, None, uc, vc, wc, h, dt)
    np.testing.assert_allclose(wc - wn3, 0.1 * (wc - wn), rtol=1e-13, atol=1e-15)


def test_cell_correction_agrees_with_face_projection():
    """The cell correction is the face-to-cell average of the face projection's
    correction: (u_f - P.project(u_f))_{f->c} == uhat_c - correct_cell_velocity(uhat_c)
    for pt = 0, on a grid with density jumps."""
    case = W.random_small_case(9, 6, 5, 8)
    rho = P.density_from_fraction(case.alpha)
    p = np.random.default_rng(3).standard_normal(rho.shape)
    un, vn, wn = P.project(rho, p, case.u, case.v, case.w, case.h, dt=0.3)
    du, dv, dw = case.u - un, case.v - vn, case.w - wn
    du[:, :, -1] = 0.0
    dv[:, -1, :] = 0.0
    ax, ay, az = P.face_to_cell(du, dv, dw)
    zero = np.zeros_like(rho)
    cu, cv, cw = P.correct_cell_velocity(rho, p, None, zero, zero, zero, case.h, dt=0.3)
    np.testing.assert_allclose(-cu, ax, rtol=0, atol=1e-12 * np.abs(ax).max())
    np.testing.assert_allclose(-cv, ay, rtol=0, atol=1e-12 * np.abs(ay).max())
    np.testing.assert_allclose(-cw, az, rtol=0, atol=1e-12 * np.abs(az).max())
