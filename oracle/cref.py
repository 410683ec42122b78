"""ctypes binding of ppref.c (plain C + OpenMP float64 reference).

TEST INFRASTRUCTURE ONLY -- see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ppref.c")
_LIB = os.path.join(_HERE, "libppref.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile ppref.c with gcc (float64, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        I, Dd, Lg = ctypes.c_int, ctypes.c_double, ctypes.c_long
        L.ppref_density_from_fraction.argtypes = [Lg, _D, Dd, Dd, _D]
        L.ppref_face_coefficients.argtypes = [I, I, I, _D, _D, _D, _D]
        L.ppref_divergence.argtypes = [I, I, I, Dd, Dd, _D, _D, _D, _D]
        L.ppref_apply.argtypes = [I, I, I, Dd, _D, _D, _D]
        L.ppref_rel_residual.argtypes = [I, I, I, Dd, _D, _D, _D, _D]
        L.ppref_rel_residual.restype = Dd
        L.ppref_solve.argtypes = [I, I, I, Dd, _D, _D, _D, Dd, I, _D]
        L.ppref_solve.restype = I
        L.ppref_num_threads.restype = I
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def density_from_fraction(alpha, rho_l=1000.0, rho_g=1.2):
    a = _c64(alpha)
    out = np.empty_like(a)
    lib().ppref_density_from_fraction(a.size, _p(a), rho_l, rho_g, _p(out))
    return out


def face_coefficients(rho):
    rho = _c64(rho)
    nz, ny, nx = rho.shape
    bx, by, bz = (np.empty_like(rho) for _ in range(3))
    lib().ppref_face_coefficients(nx, ny, nz, _p(rho), _p(bx), _p(by), _p(bz))
    return bx, by, bz


def divergence(u, v, w, h, dt=1.0):
    u, v, w = _c64(u), _c64(v), _c64(w)
    nz, ny, nx = u.shape
    out = np.empty_like(u)
    lib().ppref_divergence(nx, ny, nz, h, dt, _p(u), _p(v), _p(w), _p(out))
    return out


def apply_operator(rho, p, h):
    rho, p = _c64(rho), _c64(p)
    nz, ny, nx = rho.shape
    out = np.empty_like(p)
    lib().ppref_apply(nx, ny, nz, h, _p(rho), _p(p), _p(out))
    return out


def relative_residual(rho, b, p, h):
    rho, b, p = _c64(rho), _c64(b), _c64(p)
    nz, ny, nx = rho.shape
    scratch = np.empty_like(p)
    return float(lib().ppref_rel_residual(nx, ny, nz, h, _p(rho), _p(b), _p(p), _p(scratch)))


def solve(rho, b, h, tol=1e-13, maxit=500, x0=None):
    """Reference pressure: returns (p, iterations, relative residual, seconds)."""
    rho, b = _c64(rho), _c64(b)
    nz, ny, nx = rho.shape
    p = np.zeros_like(b) if x0 is None else _c64(x0).copy()
    rr = ctypes.c_double(0.0)
    t0 = time.perf_counter()
    it = lib().ppref_solve(nx, ny, nz, h, _p(rho), _p(b), _p(p), tol, maxit, ctypes.byref(rr))
    dt = time.perf_counter() - t0
    if it < 0:
        raise MemoryError("ppref_solve: allocation failed")
    return p, it, rr.value, dt


def num_threads() -> int:
    return int(lib().ppref_num_threads())
