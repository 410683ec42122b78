"""The C-ABI library builds, loads and exports every declared symbol (no GPU needed)."""
import os
import re
import subprocess

import pytest

from paper_2104_01636_amd import ppsolve, serve

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for hdr in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            text = re.sub(r"\(\*\w+\)\s*\(", "(", text)   # function-pointer members are not entry points
            names |= set(re.findall(r"\b(pp_[a-z_]+)\s*\(", text))
    return sorted(names)


def test_header_and_binding_agree():
    assert declared_functions() == sorted(ppsolve.EXPORTS + serve.SERVER_EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ppsolve.lib()
    out = subprocess.run(["nm", "-D", "--defined-only", ppsolve.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s(pp_[a-z_]+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)
    assert ppsolve.lib().pp_version().decode().startswith("ppsolve")


def test_footprint_is_host_only_and_validates():
    fp64 = ppsolve.footprint_bytes(256, 256, 512, "fp64")
    fp32 = ppsolve.footprint_bytes(256, 256, 512, "fp32_refined")
    n = 256 * 256 * 512
    assert 60 * n < fp64 < 130 * n          # stored face weights, Krylov vectors, coarse levels
    assert 40 * n < fp32 < 130 * n         # float64 Krylov vectors plus a float32 hierarchy
    assert ppsolve.footprint_bytes(32, 32, 63) == 0     # odd nz
    assert ppsolve.footprint_bytes(1, 32, 64) == 0      # nx < 2
    assert ppsolve.footprint_bytes(32, 32, 64, tol=0.0) == 0
    small = ppsolve.footprint_bytes(32, 32, 64)
    assert small < fp64 / 100


def test_create_rejects_bad_config_without_gpu():
    cfg = ppsolve.make_config(32, 32, 63)
    import ctypes
    h = ctypes.c_void_p()
    rc = ppsolve.lib().pp_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert rc == ppsolve.PP_ERR_INVALID and not h.value
    assert b"even" in ppsolve.lib().pp_last_error(None)


def test_grid_beyond_32_bit_indices_is_rejected():
    """Cells are indexed with 32-bit ints: a grid whose last index plus one plane
    does not fit (2^31 cells here) is refused before anything is allocated."""
    import ctypes
    for shape in [(1024, 1024, 2048), (2048, 2048, 512)]:
        assert ppsolve.footprint_bytes(*shape) == 0
        cfg = ppsolve.make_config(*shape)
        h = ctypes.c_void_p()
        rc = ppsolve.lib().pp_create(ctypes.byref(cfg), None, ctypes.byref(h))
        assert rc == ppsolve.PP_ERR_INVALID and not h.value
        assert b"32-bit" in ppsolve.lib().pp_last_error(None)
