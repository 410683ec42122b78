"""Plain definitions of the multigrid pieces, for one-by-one kernel checks.

TEST INFRASTRUCTURE ONLY -- see the package docstring.

The paper solves its pressure equations by red-black SOR relaxation,
accelerated by multigrid (Section 2.1, after eq. ppe_surface_tension), and
gives no further detail.  The pieces below are the plain definitions of the
relaxation and of the grid transfers, written without any blocking, fusion or
reordering.  They define iterates of the preconditioner only; the solution of
the pressure equation does not depend on them.

Notation: the equation on every level is K x = f with the positive
semi-definite operator

    (K x)_c = D_c x_c - sum_f W_f x_nb(f),     D_c = sum_f W_f,

summed over the six faces f of cell c (walls carry W = 0).  On the finest
level W_f = beta_f = 2/(rho_L + rho_R), so K = -h^2 A with A the operator of
step 11.  Face arrays W = (Wx, Wy, Wz) use the layout of ``poisson``.
"""
from __future__ import annotations

import numpy as np

from .poisson import face_coefficients


def fine_weights(rho):
    """Face weights of the finest level: the face coefficients beta_f."""
    return face_coefficients(rho)


def apply_k(W, x):
    """(K x)_c = D_c x_c - sum_f W_f x_nb(f)."""
    Wx, Wy, Wz = W
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    fx = Wx[:, :, :-1] * (x[:, :, 1:] - x[:, :, :-1])
    y[:, :, :-1] -= fx
    y[:, :, 1:] += fx
    fy = Wy[:, :-1, :] * (x[:, 1:, :] - x[:, :-1, :])
    y[:, :-1, :] -= fy
    y[:, 1:, :] += fy
    fz = Wz * (np.roll(x, -1, axis=0) - x)
    y -= fz
    y += np.roll(fz, 1, axis=0)
    return y


def diagonal(W):
    Wx, Wy, Wz = W
    d = Wx + Wy + Wz
    d[:, :, 1:] += Wx[:, :, :-1]
    d[:, 1:, :] += Wy[:, :-1, :]
    d += np.roll(Wz, 1, axis=0)
    return d


def colour_mask(shape, colour):
    nz, ny, nx = shape
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return ((i + j + k) & 1) == colour


def neighbour_sum(W, x):
    """sum_f W_f x_nb(f) for every cell."""
    return diagonal(W) * x - apply_k(W, x)


def rb_halfsweep(W, x, f, colour, omega=1.0):
    """One SOR half-sweep over the cells of one colour ((i+j+k) mod 2 == colour):

        x_c <- (1 - omega) x_c + omega (sum_f W_f x_nb(f) + f_c) / D_c.

    Cells of one colour only have neighbours of the other colour (nz even), so
    the half-sweep is the same in any visiting order.
    """
    x = np.array(x, dtype=np.float64, copy=True)
    m = colour_mask(x.shape, colour)
    gs = (neighbour_sum(W, x) + f) / diagonal(W)
    x[m] = (1.0 - omega) * x[m] + omega * gs[m]
    return x


def rb_halfsweep_sequential(W, x, f, colour, omega=1.0):
    """The same half-sweep, visiting the cells one at a time in lexicographic
    order and updating in place (the textbook Gauss-Seidel loop)."""
    Wx, Wy, Wz = W
    x = np.array(x, dtype=np.float64, copy=True)
    nz, ny, nx = x.shape
    for k in range(nz):
        km, kp = (k - 1) % nz, (k + 1) % nz
        for j in range(ny):
            for i in range(nx):
                if (i + j + k) & 1 != colour:
                    continue
                s = 0.0
                d = 0.0
                if i > 0:
                    s += Wx[k, j, i - 1] * x[k, j, i - 1]; d += Wx[k, j, i - 1]
                if i < nx - 1:
                    s += Wx[k, j, i] * x[k, j, i + 1]; d += Wx[k, j, i]
                if j > 0:
                    s += Wy[k, j - 1, i] * x[k, j - 1, i]; d += Wy[k, j - 1, i]
                if j < ny - 1:
                    s += Wy[k, j, i] * x[k, j + 1, i]; d += Wy[k, j, i]
                s += Wz[km, j, i] * x[km, j, i]; d += Wz[km, j, i]
                s += Wz[k, j, i] * x[kp, j, i]; d += Wz[k, j, i]
                x[k, j, i] = (1.0 - omega) * x[k, j, i] + omega * (s + f[k, j, i]) / d
    return x


def coarsen_weights(W):
    """Coarse face weight = sum of the four fine face weights that make up the
    coarse face.  With injection prolongation P and sum restriction P^T this is
    exactly K_coarse = P^T K P."""
    Wx, Wy, Wz = W
    nz, ny, nx = Wx.shape
    cx = Wx[:, :, 1::2]
    cx = cx[:, 0::2, :] + cx[:, 1::2, :]
    cx = cx[0::2] + cx[1::2]
    cy = Wy[:, 1::2, :]
    cy = cy[:, :, 0::2] + cy[:, :, 1::2]
    cy = cy[0::2] + cy[1::2]
    cz = Wz[1::2]
    cz = cz[:, :, 0::2] + cz[:, :, 1::2]
    cz = cz[:, 0::2, :] + cz[:, 1::2, :]
    return cx, cy, cz


def restrict_sum(r):
    """Coarse value = sum of the 8 fine children (P^T r)."""
    r = np.asarray(r, dtype=np.float64)
    s = r[:, :, 0::2] + r[:, :, 1::2]
    s = s[:, 0::2, :] + s[:, 1::2, :]
    return s[0::2] + s[1::2]


def prolong_inject(e):
    """Fine value = value of the parent coarse cell (P e)."""
    e = np.asarray(e, dtype=np.float64)
    return np.repeat(np.repeat(np.repeat(e, 2, axis=0), 2, axis=1), 2, axis=2)
