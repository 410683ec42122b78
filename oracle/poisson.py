"""The discrete pressure problem written out plainly (float64 numpy).

TEST INFRASTRUCTURE ONLY -- see the package docstring.

What is computed (Kumar & Vanka, arXiv 2104.01636):

* mixture density from the volume fraction -- Section 2.1, eq. (density_viscosity):
  rho = alpha_l rho_l + (1 - alpha_l) rho_g.  The inputs here carry the GAS
  fraction a = 1 - alpha_l, so rho = rho_l (1 - a) + rho_g a.
* face coefficient 1/rho_f with rho_f the linear average of the two cell
  densities -- Section 2.2, the note after the step list (cell-to-face values by
  linear averaging), giving beta_f = 2 / (rho_L + rho_R).
* boundary conditions -- Section 4: no-penetration walls in x and y (no flux
  through wall faces), periodic in z.
* pressure equation -- Section 2.2, step 11: div(grad(p) / rho) = div(u_f) / dt,
  discretised on the cells with face gradients and a face divergence.

Array layout: numpy shape (nz, ny, nx), flat index i + nx*(j + ny*k).  Face
arrays have the same shape; entry c is the +x / +y / +z face of cell c, the
z-face of the last plane joins plane 0, and the +x face of i = nx-1 and the +y
face of j = ny-1 are walls (zero gradient, ignored velocity).
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft

RHO_LIQUID = 1000.0   # Section 4: liquid density, kg/m^3
RHO_GAS = 1.2         # Section 4: gas density, kg/m^3


def density_from_fraction(alpha_gas, rho_l=RHO_LIQUID, rho_g=RHO_GAS):
    """Mixture density, eq. (density_viscosity), with the gas fraction as input."""
    a = np.asarray(alpha_gas, dtype=np.float64)
    return rho_l * (1.0 - a) + rho_g * a


def face_coefficients(rho):
    """1/rho on faces: beta_f = 2/(rho_L + rho_R); zero on wall faces; periodic in z."""
    rho = np.asarray(rho, dtype=np.float64)
    bx = np.zeros_like(rho)
    by = np.zeros_like(rho)
    bx[:, :, :-1] = 2.0 / (rho[:, :, :-1] + rho[:, :, 1:])
    by[:, :-1, :] = 2.0 / (rho[:, :-1, :] + rho[:, 1:, :])
    bz = 2.0 / (rho + np.roll(rho, -1, axis=0))
    return bx, by, bz


def gradient(p, h):
    """Face-normal gradient (p_R - p_L)/h on every face; zero on the wall faces."""
    p = np.asarray(p, dtype=np.float64)
    gx = np.zeros_like(p)
    gy = np.zeros_like(p)
    gx[:, :, :-1] = (p[:, :, 1:] - p[:, :, :-1]) / h
    gy[:, :-1, :] = (p[:, 1:, :] - p[:, :-1, :]) / h
    gz = (np.roll(p, -1, axis=0) - p) / h
    return gx, gy, gz


def divergence(u, v, w, h, dt=1.0):
    """Cell divergence of a face field divided by dt.

    Per cell: (((u_e - u_w) + (v_n - v_s)) + (w_t - w_b)) / (h*dt), where the
    west/south faces at i = 0 / j = 0 and the east/north faces at i = nx-1 /
    j = ny-1 are walls carrying zero.
    """
    u = np.array(u, dtype=np.float64, copy=True)
    v = np.array(v, dtype=np.float64, copy=True)
    w = np.asarray(w, dtype=np.float64)
    u[:, :, -1] = 0.0
    v[:, -1, :] = 0.0
    du = u.copy()
    du[:, :, 1:] -= u[:, :, :-1]
    dv = v.copy()
    dv[:, 1:, :] -= v[:, :-1, :]
    dw = w - np.roll(w, 1, axis=0)
    return ((du + dv) + dw) / (h * dt)


def apply_operator(rho, p, h):
    """A p = div(beta grad p): the left-hand side of step 11."""
    bx, by, bz = face_coefficients(rho)
    gx, gy, gz = gradient(p, h)
    return divergence(bx * gx, by * gy, bz * gz, h)


def remove_mean(b):
    b = np.asarray(b, dtype=np.float64)
    return b - b.mean()


def relative_residual(rho, b, p, h):
    """||bbar - A p||_2 / ||bbar||_2 with bbar = b - mean(b): the acceptance number."""
    bb = remove_mean(b)
    r = bb - apply_operator(rho, p, h)
    return float(np.linalg.norm(r.ravel()) / np.linalg.norm(bb.ravel()))


def relative_linf_error(p, p_ref):
    """||p - p_ref||_inf / ||p_ref||_inf after removing both means."""
    a = remove_mean(p)
    b = remove_mean(p_ref)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def assemble_dense(rho, h):
    """Dense matrix of A, column by column (small grids only)."""
    shape = np.shape(rho)
    n = int(np.prod(shape))
    if n > 4096:
        raise ValueError("dense assembly is for tiny grids")
    A = np.empty((n, n))
    e = np.zeros(n)
    for c in range(n):
        e[c] = 1.0
        A[:, c] = apply_operator(rho, e.reshape(shape), h).ravel()
        e[c] = 0.0
    return A


def solve_dense(rho, b, h):
    """Brute force: the bordered system [[A, 1], [1^T, 0]] [p; lam] = [bbar; 0]."""
    shape = np.shape(rho)
    n = int(np.prod(shape))
    A = assemble_dense(rho, h)
    M = np.zeros((n + 1, n + 1))
    M[:n, :n] = A
    M[:n, n] = 1.0
    M[n, :n] = 1.0
    rhs = np.zeros(n + 1)
    rhs[:n] = remove_mean(b).ravel()
    sol = np.linalg.solve(M, rhs)
    return sol[:n].reshape(shape)


def spectral_eigenvalues(nx, ny, nz, h):
    """Eigenvalues of the constant-coefficient operator (unit coefficient):
    cosine modes in x and y (walls), Fourier modes in z (periodic)."""
    lx = -4.0 / h ** 2 * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2
    ly = -4.0 / h ** 2 * np.sin(np.pi * np.arange(ny) / (2 * ny)) ** 2
    lz = -4.0 / h ** 2 * np.sin(np.pi * np.arange(nz) / nz) ** 2
    return lz[:, None, None] + ly[None, :, None] + lx[None, None, :]


def solve_spectral(rho0, b, h):
    """Uniform density rho0: A = L/rho0 is diagonalised by DCT-II in x, y and the
    FFT in z; the zero mode (the constants) is dropped."""
    b = remove_mean(b)
    nz, ny, nx = b.shape
    lam = spectral_eigenvalues(nx, ny, nz, h) / rho0
    bh = sfft.dctn(b, type=2, axes=(1, 2), norm="ortho")
    bh = sfft.fft(bh, axis=0)
    lam[0, 0, 0] = 1.0
    ph = bh / lam
    ph[0, 0, 0] = 0.0
    p = sfft.ifft(ph, axis=0).real
    return sfft.idctn(p, type=2, axes=(1, 2), norm="ortho")


def cell_centres(nx, ny, nz, h):
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h,
                          (np.arange(nx) + 0.5) * h, indexing="ij")
    return x, y, z


def manufactured(nx, ny, nz, h):
    """Manufactured solution with smooth density on [0,1]^2 x [0, Lz]:

    p   = cos(pi x) cos(pi y) sin(2 pi z / Lz)     (zero normal gradient at the walls)
    rho = 2 + cos(pi x) sin(2 pi z / Lz)
    f   = div(grad(p)/rho), derived by hand:
        f = (1/rho) lap(p) - (1/rho^2) grad(rho) . grad(p)

    Returns (rho, f, p) sampled at cell centres (f and p with their means removed).
    """
    Lz = nz * h
    x, y, z = cell_centres(nx, ny, nz, h)
    kz = 2.0 * np.pi / Lz
    cx, sx = np.cos(np.pi * x), np.sin(np.pi * x)
    cy, sy = np.cos(np.pi * y), np.sin(np.pi * y)
    sz, cz = np.sin(kz * z), np.cos(kz * z)
    p = cx * cy * sz
    rho = 2.0 + cx * sz
    lap = -(2.0 * np.pi ** 2 + kz ** 2) * p
    dpx, dpy, dpz = -np.pi * sx * cy * sz, -np.pi * cx * sy * sz, kz * cx * cy * cz
    drx, dry, drz = -np.pi * sx * sz, 0.0 * x, kz * cx * cz
    f = lap / rho - (drx * dpx + dry * dpy + drz * dpz) / rho ** 2
    return rho, remove_mean(f), remove_mean(p)


def project(rho, p, u, v, w, h, dt=1.0):
    """Face-velocity correction of the projection (Section 2.2, step 12, on faces):
    u_f <- u_f - dt * beta_f * (grad p)_f; wall faces stay zero."""
    bx, by, bz = face_coefficients(rho)
    gx, gy, gz = gradient(p, h)
    un = np.array(u, dtype=np.float64, copy=True) - dt * (bx * gx)
    vn = np.array(v, dtype=np.float64, copy=True) - dt * (by * gy)
    wn = np.asarray(w, dtype=np.float64) - dt * (bz * gz)
    un[:, :, -1] = 0.0
    vn[:, -1, :] = 0.0
    return un, vn, wn


def face_to_cell(fx, fy, fz):
    """Linear average of the two faces that bound a cell along each axis (the
    face-to-cell counterpart of the linear cell-to-face averaging defined in the
    note after the step list of Section 2.2).  Face arrays use the +face layout:
    the west face of cell i is the +x face of cell i-1, and the wall faces
    (i = -1/2, i = nx-1/2 and likewise in y) carry zero; z is periodic."""
    fx = np.array(fx, dtype=np.float64, copy=True)
    fy = np.array(fy, dtype=np.float64, copy=True)
    fz = np.asarray(fz, dtype=np.float64)
    fx[:, :, -1] = 0.0
    fy[:, -1, :] = 0.0
    wx = np.zeros_like(fx)
    wx[:, :, 1:] = fx[:, :, :-1]
    sy = np.zeros_like(fy)
    sy[:, 1:, :] = fy[:, :-1, :]
    bz = np.roll(fz, 1, axis=0)
    return 0.5 * (wx + fx), 0.5 * (sy + fy), 0.5 * (bz + fz)


def correct_cell_velocity(rho, p, pt, uc, vc, wc, h, dt=1.0):
    """Step 12 of Section 2.2 on the cell-centred velocity:

        u_c <- uhat_c - dt * (grad(p)/rho + grad(pt)/rho)_{f->c}

    with the face terms beta_f (p_R - p_L)/h + beta_f (pt_R - pt_L)/h (beta_f =
    1/rho_f, rho_f the linear average; zero on the walls), averaged to the cell
    by face_to_cell.  pt (the surface-tension pressure of step 6) may be None."""
    bx, by, bz = face_coefficients(rho)
    gx, gy, gz = gradient(p, h)
    fx, fy, fz = bx * gx, by * gy, bz * gz
    if pt is not None:
        tx, ty, tz = gradient(pt, h)
        fx, fy, fz = fx + bx * tx, fy + by * ty, fz + bz * tz
    ax, ay, az = face_to_cell(fx, fy, fz)
    return (np.asarray(uc, dtype=np.float64) - dt * ax, np.asarray(vc, dtype=np.float64) - dt * ay,
            np.asarray(wc, dtype=np.float64) - dt * az)


def surface_force(alpha_gas, kappa, sigma, h):
    """Sharp-surface-force face values (Section 2.1, eq. jump_condition, with the
    jump applied at faces): f_f = sigma * kappa_f * (a_R - a_L) / h, kappa_f the
    linear average of the cell curvatures; zero on wall faces.  With this sign the
    balancing pressure is higher inside the gas (p = sigma kappa a for constant kappa)."""
    a = np.asarray(alpha_gas, dtype=np.float64)
    k = np.broadcast_to(np.asarray(kappa, dtype=np.float64), a.shape)
    fx = np.zeros_like(a)
    fy = np.zeros_like(a)
    fx[:, :, :-1] = sigma * (0.5 * (k[:, :, :-1] + k[:, :, 1:])) * ((a[:, :, 1:] - a[:, :, :-1]) / h)
    fy[:, :-1, :] = sigma * (0.5 * (k[:, :-1, :] + k[:, 1:, :])) * ((a[:, 1:, :] - a[:, :-1, :]) / h)
    kn = np.roll(k, -1, axis=0)
    fz = sigma * (0.5 * (k + kn)) * ((np.roll(a, -1, axis=0) - a) / h)
    return fx, fy, fz


def surface_tension_rhs(rho, alpha_gas, kappa, sigma, h):
    """Right-hand side of the surface-tension pressure equation (Section 2.1,
    eq. ppe_surface_tension with eq. jump_condition as the source):
    div(beta grad p~) = div(beta f)."""
    bx, by, bz = face_coefficients(rho)
    fx, fy, fz = surface_force(alpha_gas, kappa, sigma, h)
    return divergence(bx * fx, by * fy, bz * fz, h)
