"""Kernel-level parity: the finest-level passes of the multigrid cycle, element by
element against the oracle's plain definitions (needs an MI355X).

The two legs of the cycle are run through the C ABI (pp_presmooth_restrict,
pp_prolong_postsmooth) by the same kernels the preconditioner launches on the
finest level: in float64 the red sweep from zero, the black half-sweep, the
residual restriction, the prolongation with the black update and the red
half-sweep with its two dots; in float32 (refined form) the overlapped-tile
kernels that fuse them, on grids of at most 65536 or at least 2^20 cells, and
the separate passes in between.  The oracle side composes relax.rb_halfsweep,
relax.apply_k, relax.restrict_sum and relax.prolong_inject in float64 on the
same inputs (the float32 inputs upcast exactly).

Tolerances: float64, 1e-12 of the scale of the values compared (one rounding of
a sum of seven terms, and the residual's cancellation against f); float32,
2e-5 of that scale (the weights formed in float32 from the float32 density with
the hardware reciprocal, about 2e-7 each, through two dependent half-sweeps).
"""
import numpy as np
import pytest
import torch

from oracle import poisson as P, relax as R
from paper_2104_01636_amd import ppsolve, workload as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"fp64": 1e-12, "fp32_refined": 2e-5}
NP = {"fp64": np.float64, "fp32_refined": np.float32}


def say(*a):
    print(*a, flush=True)


def to_dev(a, dtype=np.float64):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


# (nz, ny, nx): grids that coarsen; 32x32x64 and 256x256x512 run the fused float32
# kernels, 64x64x128 (524288 cells) their unfused passes; rows of 256, 128 and 64
# cells run the row-wave forms of the fused kernels (a wavefront per row; with 64,
# one cell per lane and the x pairs across lane pairs), here with a partial last
# band of rows
SHAPES = [(8, 6, 10), (12, 10, 6), (16, 8, 8), (64, 32, 32), (128, 64, 64), (8, 10, 256), (16, 24, 128),
          (16, 22, 64)]


def case_for(shape, seed):
    nz, ny, nx = shape
    if shape == (512, 256, 256):
        return W.preset("duct256")
    return W.random_small_case(seed, nx, ny, nz)


def inputs(case, mode, seed):
    rng = np.random.default_rng(seed)
    rho = P.density_from_fraction(case.alpha)
    b = P.divergence(case.u, case.v, case.w, case.h)
    f = (-case.h ** 2 * (b - b.mean())).astype(NP[mode])   # the cycle's scaled right-hand side
    return rho, f.astype(np.float64), rng


@pytest.mark.parametrize("shape", SHAPES + [(512, 256, 256)])
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_presmooth_restrict_matches_definitions(shape, mode):
    nz, ny, nx = shape
    say("presmooth_restrict", shape, mode)
    case = case_for(shape, 100 + sum(shape))
    rho, f, _ = inputs(case, mode, 1)
    Wt = R.fine_weights(rho)
    x_ref = R.rb_halfsweep(Wt, np.zeros_like(f), f, 0)
    x_ref = R.rb_halfsweep(Wt, x_ref, f, 1)
    r_ref = f - R.apply_k(Wt, x_ref)
    rc_ref = R.restrict_sum(r_ref)
    with ppsolve.Solver(nx, ny, nz, case.h, mode=mode) as S:
        S.set_density(to_dev(rho))
        x, rc = S.presmooth_restrict(to_dev(f, NP[mode]))
        x, rc = host(x), host(rc)
    sx = np.abs(x_ref).max()
    sr = np.abs(f).max() + np.abs(R.diagonal(Wt)).max() * sx
    ex, er = np.abs(x - x_ref).max() / sx, np.abs(rc - rc_ref).max() / (8 * sr)
    say(f"   x err {ex:.2e}  rc err {er:.2e}")
    assert ex <= TOL[mode] and er <= TOL[mode]


@pytest.mark.parametrize("shape,wc", [(sh, w) for sh in SHAPES for w in (1.0, 2.0)] + [((512, 256, 256), 1.0)])
@pytest.mark.parametrize("mode", ["fp64", "fp32_refined"])
def test_prolong_postsmooth_matches_definitions(shape, mode, wc):
    nz, ny, nx = shape
    say("prolong_postsmooth", shape, mode, wc)
    case = case_for(shape, 200 + sum(shape))
    rho, f, rng = inputs(case, mode, 2)
    sf = np.abs(f).max()
    x = (rng.standard_normal(f.shape) * sf).astype(NP[mode]).astype(np.float64)
    e = (rng.standard_normal((nz // 2, ny // 2, nx // 2)) * sf).astype(NP[mode]).astype(np.float64)
    q = rng.standard_normal(f.shape)
    Wt = R.fine_weights(rho)
    y = x + wc * R.prolong_inject(e)
    y = R.rb_halfsweep(Wt, y, f, 1)
    z_ref = R.rb_halfsweep(Wt, y, f, 0)
    with ppsolve.Solver(nx, ny, nz, case.h, mode=mode) as S:
        S.set_density(to_dev(rho))
        z = host(S.prolong_postsmooth(to_dev(f, NP[mode]), to_dev(x, NP[mode]), to_dev(e, NP[mode]), wc))
        z2, (sz, zq) = S.prolong_postsmooth(to_dev(f, NP[mode]), to_dev(x, NP[mode]), to_dev(e, NP[mode]), wc,
                                           q=to_dev(q))
        z2 = host(z2)
    np.testing.assert_array_equal(z2, z)     # the reducing variant writes the same values
    s = np.abs(z_ref).max()
    err = np.abs(z - z_ref).max() / s
    say(f"   z err {err:.2e}")
    assert err <= TOL[mode]
    # the two dots of the pass: sum(z) and <z, q>, against the oracle's z
    assert abs(sz - z_ref.sum()) <= TOL[mode] * np.abs(z_ref).sum()
    assert abs(zq - np.sum(z_ref * q)) <= TOL[mode] * np.sum(np.abs(z_ref * q))
    # and bit-consistent with the z the pass wrote (float64 sums in a fixed order)
    assert sz == pytest.approx(z.sum(), rel=1e-9, abs=1e-12 * np.abs(z).sum())


def test_cycle_legs_reject_grids_that_do_not_coarsen():
    case = W.random_small_case(7, 6, 5, 4)   # ny odd
    rho = P.density_from_fraction(case.alpha)
    with ppsolve.Solver(6, 5, 4, case.h) as S:
        f = torch.zeros((4, 5, 6), dtype=torch.float64, device=DEV)
        with pytest.raises(ppsolve.PPError) as e:
            S.presmooth_restrict(f)
        assert e.value.code == ppsolve.PP_ERR_STATE
        S.set_density(to_dev(rho))
        with pytest.raises(ppsolve.PPError) as e:
            S.presmooth_restrict(f)
        assert e.value.code == ppsolve.PP_ERR_INVALID
