"""Python side of the serving loop (include/pp_server.h): ctypes wrapper and a
real-time replay driver for a stream of solve requests.

The scheduler, admission, residency and concurrency are in the library (C++);
this module only marshals arguments and replays arrival times.
"""
from __future__ import annotations

import ctypes
import threading
import time

from . import ppsolve
from .ppsolve import Config, Stats, lib

_vp = ctypes.c_void_p
FOOTPRINT_FN = ctypes.CFUNCTYPE(ctypes.c_size_t, _vp, ctypes.POINTER(Config))
OPEN_FN = ctypes.CFUNCTYPE(ctypes.c_int, _vp, ctypes.POINTER(Config), ctypes.POINTER(_vp))
SETRHO_FN = ctypes.CFUNCTYPE(ctypes.c_int, _vp, _vp, _vp)
SOLVE_FN = ctypes.CFUNCTYPE(ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.POINTER(Stats))
CLOSE_FN = ctypes.CFUNCTYPE(None, _vp, _vp)
ERROR_FN = ctypes.CFUNCTYPE(_vp, _vp, _vp)  # returns the address of a NUL-terminated message


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("slots", ctypes.c_int)]


class Backend(ctypes.Structure):
    _fields_ = [("ctx", _vp), ("footprint", FOOTPRINT_FN), ("open_case", OPEN_FN), ("set_density", SETRHO_FN),
                ("solve", SOLVE_FN), ("close_case", CLOSE_FN), ("error", ERROR_FN)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("stats", Stats), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_end", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("new_density", ctypes.c_int), ("message", ctypes.c_char * 160)]

    def as_dict(self):
        return {"status": self.status, "stats": self.stats.as_dict(), "t_submit": self.t_submit,
                "t_start": self.t_start, "t_end": self.t_end, "latency_ms": self.latency_ms,
                "new_density": bool(self.new_density), "message": self.message.decode()}


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_longlong), ("succeeded", ctypes.c_longlong), ("rejected", ctypes.c_longlong),
                ("queued", ctypes.c_longlong), ("running", ctypes.c_int), ("max_running", ctypes.c_int),
                ("resident_cases", ctypes.c_longlong), ("resident_bytes", ctypes.c_size_t),
                ("peak_resident_bytes", ctypes.c_size_t), ("evictions", ctypes.c_longlong),
                ("latency_p50_ms", ctypes.c_double), ("latency_p99_ms", ctypes.c_double),
                ("latency_max_ms", ctypes.c_double), ("solves_per_s", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _bind():
    L = lib()
    if getattr(L, "_srv_bound", False):
        return L
    L.pp_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(Backend), ctypes.POINTER(_vp)]
    L.pp_server_create.restype = ctypes.c_int
    L.pp_server_submit.argtypes = [_vp, ctypes.c_longlong, ctypes.POINTER(Config), _vp, _vp, _vp,
                                   ctypes.POINTER(ctypes.c_longlong)]
    L.pp_server_submit.restype = ctypes.c_int
    L.pp_server_wait.argtypes = [_vp, ctypes.c_longlong, ctypes.c_double, ctypes.POINTER(RequestResult)]
    L.pp_server_wait.restype = ctypes.c_int
    L.pp_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.pp_server_get_stats.restype = ctypes.c_int
    L.pp_server_destroy.argtypes = [_vp]
    L.pp_server_destroy.restype = ctypes.c_int
    L.pp_server_last_error.restype = ctypes.c_char_p
    L._srv_bound = True
    return L


SERVER_EXPORTS = ("pp_server_create", "pp_server_submit", "pp_server_wait", "pp_server_get_stats",
                  "pp_server_destroy", "pp_server_last_error")


class Server:
    """pp_server: slots run concurrently, cases stay resident within budget_bytes."""

    def __init__(self, budget_bytes: int, slots: int = 4, backend: Backend | None = None):
        L = _bind()
        self._cfg = ServerConfig(int(budget_bytes), int(slots))
        self._backend = backend  # keep callbacks alive
        self._s = _vp()
        rc = L.pp_server_create(ctypes.byref(self._cfg), ctypes.byref(backend) if backend is not None else None,
                                ctypes.byref(self._s))
        if rc != 0:
            raise ppsolve.PPError(rc, L.pp_server_last_error().decode())

    def submit(self, case_id: int, cfg: Config, rho_ptr, rhs_ptr, p_out_ptr) -> int:
        rid = ctypes.c_longlong()
        rc = _bind().pp_server_submit(self._s, int(case_id), ctypes.byref(cfg), rho_ptr, rhs_ptr, p_out_ptr,
                                      ctypes.byref(rid))
        if rc != 0:
            raise ppsolve.PPError(rc, _bind().pp_server_last_error().decode())
        return rid.value

    def wait(self, req_id: int, timeout_s: float = -1.0) -> dict | None:
        out = RequestResult()
        rc = _bind().pp_server_wait(self._s, int(req_id), float(timeout_s), ctypes.byref(out))
        if rc == 1:
            return None
        if rc != 0:
            raise ppsolve.PPError(rc, _bind().pp_server_last_error().decode())
        return out.as_dict()

    def stats(self) -> dict:
        out = ServerStats()
        _bind().pp_server_get_stats(self._s, ctypes.byref(out))
        return out.as_dict()

    def close(self):
        if self._s:
            _bind().pp_server_destroy(self._s)
            self._s = _vp()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def replay(server: Server, requests, time_scale: float = 1.0):
    """Submit each request at its arrival time (seconds from now, scaled) from a
    separate thread and wait for all results.

    requests: list of dicts with keys arrival_s, case_id, cfg (Config), rho, rhs,
    p_out (device pointers or None).  Returns the list of result dicts (in order).
    """
    ids = [None] * len(requests)
    t0 = time.perf_counter()

    def feeder():
        for i, r in enumerate(requests):
            delay = t0 + r["arrival_s"] * time_scale - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            ids[i] = server.submit(r["case_id"], r["cfg"], r["rho"], r["rhs"], r["p_out"])

    th = threading.Thread(target=feeder, daemon=True)
    th.start()
    th.join()
    return [server.wait(i) for i in ids]
