"""pp_rel_residual_noalloc through the C ABI against pp_rel_residual (needs an MI355X).

Both run the same kernels and fixed-order reductions, the no-allocation entry
point on its static per-GPU scratch array: the results must be bit-identical,
on two calls in a row (the second with a smaller grid, so stale partial sums of
the first would show), and a grid needing more partial sums than the array holds
is refused before any work.
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import cref, poisson as P
from paper_2104_01636_amd import ppsolve, workload as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def noalloc(rho, b, p, h):
    nz, ny, nx = rho.shape
    out = ctypes.c_double(-1.0)
    rc = ppsolve.lib().pp_rel_residual_noalloc(nx, ny, nz, float(h), ctypes.c_void_p(rho.data_ptr()),
                                               ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(p.data_ptr()),
                                               ctypes.byref(out), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, out.value


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    results = []
    for shape, seed in [((64, 32, 48), 1), ((6, 5, 7), 2)]:     # second call smaller
        nz, ny, nx = shape
        case = W.random_small_case(500 + seed, nx, ny, nz)
        rho = gpu(P.density_from_fraction(case.alpha))
        b = gpu(P.divergence(case.u, case.v, case.w, case.h) + 0.5)
        p = gpu(np.random.default_rng(seed).standard_normal(shape))
        rc, got = noalloc(rho, b, p, case.h)
        assert rc == ppsolve.PP_OK, ppsolve.lib().pp_last_error(None)
        want = ppsolve.rel_residual(rho, b, p, case.h)
        assert got == want                                      # same kernels, same order: bit-identical
        ref = cref.relative_residual(rho.cpu().numpy(), b.cpu().numpy(), p.cpu().numpy(), case.h)
        assert got == pytest.approx(ref, rel=1e-12)
        results.append(got)
    assert results[0] != results[1]


def test_noalloc_rejects_grids_beyond_its_scratch():
    t = torch.zeros(8, dtype=torch.float64, device=DEV)
    out = ctypes.c_double()
    # 8192 x 512 cells per plane: 128 x 64 tiles of 64 x 8, more partial sums than the scratch holds
    rc = ppsolve.lib().pp_rel_residual_noalloc(8192, 512, 2, 1.0, ctypes.c_void_p(t.data_ptr()),
                                               ctypes.c_void_p(t.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                               ctypes.byref(out), None)
    assert rc == ppsolve.PP_ERR_INVALID
    assert b"4096 tiles" in ppsolve.lib().pp_last_error(None)
