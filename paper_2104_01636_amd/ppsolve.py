"""ctypes binding of libppsolve.so (include/pp.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  torch supplies device memory and the stream.  If the library is
missing this module raises on first use -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppsolve.so")

PP_OK = 0
PP_ERR_INVALID = -1
PP_ERR_OOM = -2
PP_ERR_NOT_CONVERGED = -3
PP_ERR_HIP = -4
PP_ERR_NONFINITE = -5
PP_ERR_STATE = -6
_NAMES = {0: "PP_OK", -1: "PP_ERR_INVALID", -2: "PP_ERR_OOM", -3: "PP_ERR_NOT_CONVERGED", -4: "PP_ERR_HIP",
          -5: "PP_ERR_NONFINITE", -6: "PP_ERR_STATE"}

MODES = {"fp64": 0, "fp32_refined": 1}

# Every entry point declared in include/pp.h.
EXPORTS = ("pp_footprint_bytes", "pp_create", "pp_set_density", "pp_solve", "pp_apply", "pp_presmooth_restrict",
           "pp_prolong_postsmooth", "pp_destroy",
           "pp_last_error", "pp_density_from_fraction", "pp_divergence", "pp_project", "pp_correct_velocity",
           "pp_surface_tension_rhs",
           "pp_rel_residual", "pp_rel_residual_noalloc", "pp_kernel_timing", "pp_version")


class PPError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_NAMES.get(code, code)}: {message}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("h", ctypes.c_double),
                ("mode", ctypes.c_int), ("tol", ctypes.c_double), ("max_iters", ctypes.c_int),
                ("pre_sweeps", ctypes.c_int), ("post_sweeps", ctypes.c_int), ("flags", ctypes.c_int),
                ("omega", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("total_ms", ctypes.c_double), ("launches", ctypes.c_longlong),
                ("bytes", ctypes.c_double)]


_lib = None


def lib():
    """Load the library (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2104_01636_amd/build.py "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        vp, cd, ci, sz = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
        L.pp_footprint_bytes.argtypes = [ctypes.POINTER(Config)]
        L.pp_footprint_bytes.restype = sz
        L.pp_create.argtypes = [ctypes.POINTER(Config), vp, ctypes.POINTER(vp)]
        L.pp_set_density.argtypes = [vp, vp]
        L.pp_solve.argtypes = [vp, vp, vp, ctypes.POINTER(Stats)]
        L.pp_apply.argtypes = [vp, vp, vp]
        L.pp_presmooth_restrict.argtypes = [vp, vp, vp, vp]
        L.pp_prolong_postsmooth.argtypes = [vp, vp, vp, vp, cd, vp, vp, ctypes.POINTER(ctypes.c_double)]
        L.pp_destroy.argtypes = [vp]
        L.pp_last_error.argtypes = [vp]
        L.pp_last_error.restype = ctypes.c_char_p
        L.pp_density_from_fraction.argtypes = [vp, cd, cd, vp, sz, vp]
        L.pp_divergence.argtypes = [ci, ci, ci, cd, cd, vp, vp, vp, vp, vp]
        L.pp_version.restype = ctypes.c_char_p
        L.pp_project.argtypes = [ci, ci, ci, cd, cd, vp, vp, vp, vp, vp, vp]
        L.pp_surface_tension_rhs.argtypes = [ci, ci, ci, cd, cd, vp, vp, vp, vp, vp]
        L.pp_correct_velocity.argtypes = [ci, ci, ci, cd, cd, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.pp_correct_velocity.restype = ci
        L.pp_rel_residual.argtypes = [ci, ci, ci, cd, vp, vp, vp, ctypes.POINTER(cd), vp]
        L.pp_rel_residual.restype = ci
        L.pp_rel_residual_noalloc.argtypes = [ci, ci, ci, cd, vp, vp, vp, ctypes.POINTER(cd), vp]
        L.pp_rel_residual_noalloc.restype = ci
        L.pp_kernel_timing.argtypes = [vp, ci, ctypes.POINTER(KernelTime), ci]
        L.pp_kernel_timing.restype = ci
        for name in ("pp_create", "pp_set_density", "pp_solve", "pp_apply", "pp_presmooth_restrict",
                     "pp_prolong_postsmooth", "pp_destroy",
                     "pp_density_from_fraction", "pp_divergence", "pp_project", "pp_surface_tension_rhs"):
            getattr(L, name).restype = ci
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    if rc != PP_OK:
        msg = lib().pp_last_error(handle).decode()
        raise PPError(rc, msg)


PP_FLAG_MG_SOLVER = 1
PP_FLAG_W_CYCLE = 2


def make_config(nx, ny, nz, h=None, mode="fp64", tol=1e-10, max_iters=1000, pre_sweeps=0, post_sweeps=0, flags=0,
                omega=0.0):
    return Config(int(nx), int(ny), int(nz), float(h if h is not None else 1.0 / nx), MODES[mode] if isinstance(mode, str)
                  else int(mode), float(tol), int(max_iters), int(pre_sweeps), int(post_sweeps), int(flags),
                  float(omega))


def footprint_bytes(nx, ny, nz, mode="fp64", **kw) -> int:
    cfg = make_config(nx, ny, nz, mode=mode, **kw)
    return int(lib().pp_footprint_bytes(ctypes.byref(cfg)))


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, n: int, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One pressure-solver handle (pp_create ... pp_destroy)."""

    def __init__(self, nx, ny, nz, h=None, mode="fp64", tol=1e-10, max_iters=1000, stream=None, **kw):
        self.cfg = make_config(nx, ny, nz, h, mode, tol, max_iters, **kw)
        self.n = int(nx) * int(ny) * int(nz)
        self.shape = (int(nz), int(ny), int(nx))
        self.stream = stream
        self._h = ctypes.c_void_p()
        _check(lib().pp_create(ctypes.byref(self.cfg), _stream_ptr(stream), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def set_density(self, rho: torch.Tensor):
        _check(lib().pp_set_density(self._h, _dev(rho, self.n, "rho")), self._h)

    def solve(self, rhs: torch.Tensor, p: torch.Tensor | None = None, check=True):
        if p is None:
            p = torch.zeros(self.shape, dtype=torch.float64, device=rhs.device)
        st = Stats()
        rc = lib().pp_solve(self._h, _dev(rhs, self.n, "rhs"), _dev(p, self.n, "p"), ctypes.byref(st))
        if check:
            _check(rc, self._h)
        return p, st.as_dict() | {"status": rc}

    def apply(self, x: torch.Tensor, y: torch.Tensor | None = None):
        if y is None:
            y = torch.empty_like(x)
        _check(lib().pp_apply(self._h, _dev(x, self.n, "x"), _dev(y, self.n, "y")), self._h)
        return y

    @property
    def cycle_dtype(self):
        """Precision of the multigrid cycle's arrays (float64, or float32 in the refined form)."""
        return torch.float64 if self.cfg.mode == MODES["fp64"] else torch.float32

    def _cyc(self, t: torch.Tensor, n: int, name: str):
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.cycle_dtype:
            raise TypeError(f"{name} must be a {self.cycle_dtype} CUDA tensor")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name} must be contiguous with {n} elements")
        return ctypes.c_void_p(t.data_ptr())

    def _coarse_n(self):
        nz, ny, nx = self.shape
        return (nz // 2) * (ny // 2) * (nx // 2)

    def presmooth_restrict(self, f: torch.Tensor):
        """Down leg of the finest-level cycle: returns (x, rc)."""
        nz, ny, nx = self.shape
        x = torch.empty_like(f)
        rc = torch.empty((nz // 2, ny // 2, nx // 2), dtype=f.dtype, device=f.device)
        _check(lib().pp_presmooth_restrict(self._h, self._cyc(f, self.n, "f"), self._cyc(x, self.n, "x"),
                                           self._cyc(rc, rc.numel(), "rc")), self._h)
        return x, rc

    def prolong_postsmooth(self, f: torch.Tensor, x: torch.Tensor, e: torch.Tensor, wc: float = 1.0,
                           q: torch.Tensor | None = None):
        """Up leg of the finest-level cycle: returns z, or (z, (sum z, <z, q>)) with q."""
        z = torch.empty_like(f)
        dots = (ctypes.c_double * 2)()
        _check(lib().pp_prolong_postsmooth(self._h, self._cyc(f, self.n, "f"), self._cyc(x, self.n, "x"),
                                           self._cyc(e, self._coarse_n(), "e"), float(wc), self._cyc(z, self.n, "z"),
                                           _dev(q, self.n, "q") if q is not None else None,
                                           dots if q is not None else None), self._h)
        return (z, (dots[0], dots[1])) if q is not None else z

    def timing(self, mode: int):
        """mode 1: start (clear), -1: stop, 0: return {name: (total_ms, launches, bytes)}."""
        if mode != 0:
            rc = lib().pp_kernel_timing(self._h, mode, None, 0)
            if rc < 0:
                _check(rc, self._h)
            return None
        buf = (KernelTime * 64)()
        n = lib().pp_kernel_timing(self._h, 0, buf, 64)
        if n < 0:
            _check(n, self._h)
        return {buf[i].name.decode(): (buf[i].total_ms, buf[i].launches, buf[i].bytes) for i in range(n)}

    def close(self):
        if self._h:
            lib().pp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def density_from_fraction(alpha: torch.Tensor, rho_l=1000.0, rho_g=1.2, out=None, stream=None):
    n = alpha.numel()
    out = torch.empty_like(alpha) if out is None else out
    _check(lib().pp_density_from_fraction(_dev(alpha, n, "alpha"), float(rho_l), float(rho_g), _dev(out, n, "rho"), n,
                                          _stream_ptr(stream)))
    return out


def divergence(u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, h: float, dt: float = 1.0, out=None, stream=None):
    nz, ny, nx = u.shape
    n = u.numel()
    out = torch.empty_like(u) if out is None else out
    _check(lib().pp_divergence(nx, ny, nz, float(h), float(dt), _dev(u, n, "u"), _dev(v, n, "v"), _dev(w, n, "w"),
                               _dev(out, n, "out"), _stream_ptr(stream)))
    return out


def project(rho: torch.Tensor, p: torch.Tensor, u: torch.Tensor, v: torch.Tensor, w: torch.Tensor, h: float,
            dt: float = 1.0, stream=None):
    """In place: u, v, w -= dt * beta_f * grad(p) on faces (wall faces zeroed)."""
    nz, ny, nx = u.shape
    n = u.numel()
    _check(lib().pp_project(nx, ny, nz, float(h), float(dt), _dev(rho, n, "rho"), _dev(p, n, "p"), _dev(u, n, "u"),
                            _dev(v, n, "v"), _dev(w, n, "w"), _stream_ptr(stream)))
    return u, v, w


def correct_velocity(rho: torch.Tensor, p: torch.Tensor, pt: torch.Tensor | None, u: torch.Tensor, v: torch.Tensor,
                     w: torch.Tensor, uc: torch.Tensor, vc: torch.Tensor, wc: torch.Tensor, h: float, dt: float = 1.0,
                     stream=None):
    """Step 12 in place: face velocities projected with p, cell velocities corrected with
    (grad p / rho + grad pt / rho) averaged from faces to cells (pt may be None)."""
    nz, ny, nx = u.shape
    n = u.numel()
    _check(lib().pp_correct_velocity(nx, ny, nz, float(h), float(dt), _dev(rho, n, "rho"), _dev(p, n, "p"),
                                     _dev(pt, n, "pt") if pt is not None else None, _dev(u, n, "u"), _dev(v, n, "v"),
                                     _dev(w, n, "w"), _dev(uc, n, "uc"), _dev(vc, n, "vc"), _dev(wc, n, "wc"),
                                     _stream_ptr(stream)))
    return u, v, w, uc, vc, wc


def surface_tension_rhs(rho: torch.Tensor, alpha: torch.Tensor, kappa: torch.Tensor, sigma: float, h: float, out=None,
                        stream=None):
    nz, ny, nx = rho.shape
    n = rho.numel()
    out = torch.empty_like(rho) if out is None else out
    _check(lib().pp_surface_tension_rhs(nx, ny, nz, float(h), float(sigma), _dev(rho, n, "rho"),
                                        _dev(alpha, n, "alpha"), _dev(kappa, n, "kappa"), _dev(out, n, "out"),
                                        _stream_ptr(stream)))
    return out


@dataclass
class Result:
    p: torch.Tensor
    stats: dict


def rel_residual(rho: torch.Tensor, rhs: torch.Tensor, p: torch.Tensor, h: float, stream=None,
                 noalloc: bool = False) -> float:
    """||bbar - A p|| / ||bbar|| on the device (pp_rel_residual, or pp_rel_residual_noalloc)."""
    nz, ny, nx = rho.shape
    n = rho.numel()
    out = ctypes.c_double()
    fn = lib().pp_rel_residual_noalloc if noalloc else lib().pp_rel_residual
    _check(fn(nx, ny, nz, float(h), _dev(rho, n, "rho"), _dev(rhs, n, "rhs"), _dev(p, n, "p"), ctypes.byref(out),
              _stream_ptr(stream)))
    return out.value
