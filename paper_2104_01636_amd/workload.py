"""Seeded synthetic inputs for the pressure solve: bubble swarms and face velocities.

This module only draws random numbers and does geometry.  It computes none of
the solver's arithmetic: the mixture density rule, the divergence and the
operator live in the library (and, independently, in the CPU checker).  Both
sides consume the arrays made here.

Array layout (shared by every consumer): numpy shape ``(nz, ny, nx)``, C order,
so the flat index is ``i + nx*(j + ny*k)`` with x fastest and z (streamwise,
periodic) slowest.  Face arrays use the same shape: entry ``c`` of ``u`` is the
x-face at ``i+1/2`` of cell ``c``, of ``v`` the y-face at ``j+1/2``, of ``w``
the z-face at ``k+1/2`` (the one at ``k = nz-1`` joins cell ``k = 0``).  The
wall faces ``i = nx-1`` and ``j = ny-1`` are stored as zero; the faces at
``i = -1/2`` and ``j = -1/2`` are walls and are not stored.

Volume fraction: ``alpha`` is the GAS fraction of each cell, the number of its
4x4x4 sub-cell centres that lie strictly inside some bubble, divided by 64
(exact in float64).  Positions are in cell units: cell ``(i, j, k)`` covers
``[i, i+1) x [j, j+1) x [k, k+1)``; distances along z use the minimum image.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SUB = 4  # sub-cells per cell edge for the volume fraction
_FULL = np.uint64(0xFFFFFFFFFFFFFFFF)


@dataclass
class Case:
    """One synthetic duct case: grid, bubbles, gas fraction and face velocities."""
    nx: int
    ny: int
    nz: int
    h: float
    centres: np.ndarray          # (n, 3) float64, cell units, columns x, y, z
    diameter: float              # cells
    alpha: np.ndarray            # (nz, ny, nx) float64 gas fraction, multiples of 1/64
    u: np.ndarray = field(repr=False, default=None)
    v: np.ndarray = field(repr=False, default=None)
    w: np.ndarray = field(repr=False, default=None)
    name: str = ""
    seed: int = 0

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def _min_image(dz: np.ndarray, nz: int) -> np.ndarray:
    return dz - nz * np.round(dz / nz)


def place_bubbles(rng: np.random.Generator, nx: int, ny: int, nz: int, n: int,
                  diameter: float, min_dist: float, max_tries: int = 10_000) -> np.ndarray:
    """Dart throwing: centres uniform in x, y in [r+1, W-r-1] and z in [0, nz).

    A candidate is kept when its distance to every kept centre (minimum image in
    z) is at least ``min_dist``.  Returns the kept centres, at most ``n``; fewer
    when a bubble cannot be placed within ``max_tries`` draws.
    """
    r = 0.5 * diameter
    lo_x, hi_x = r + 1.0, nx - r - 1.0
    lo_y, hi_y = r + 1.0, ny - r - 1.0
    if hi_x < lo_x or hi_y < lo_y:
        raise ValueError(f"bubble of diameter {diameter} does not fit a {nx}x{ny} cross-section")
    kept = np.empty((n, 3))
    m = 0
    md2 = float(min_dist) ** 2
    for _ in range(n):
        ok = False
        for _t in range(max_tries):
            c = np.array([rng.uniform(lo_x, hi_x), rng.uniform(lo_y, hi_y), rng.uniform(0.0, nz)])
            if m == 0:
                ok = True
            else:
                d = kept[:m] - c
                d[:, 2] = _min_image(d[:, 2], nz)
                ok = bool(np.min(np.einsum("ij,ij->i", d, d)) >= md2)
            if ok:
                kept[m] = c
                m += 1
                break
        if not ok:
            break
    return kept[:m].copy()


def lattice_bubbles(nx: int, ny: int, nz: int, counts, spacing, offset) -> np.ndarray:
    """Centres on a regular array (counts per axis, spacing and offset in cells)."""
    gx = offset[0] + spacing[0] * np.arange(counts[0])
    gy = offset[1] + spacing[1] * np.arange(counts[1])
    gz = offset[2] + spacing[2] * np.arange(counts[2])
    zz, yy, xx = np.meshgrid(gz, gy, gx, indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.float64)


# Sub-cell centre offsets inside one cell, bit b = sx + 4*(sy + 4*sz).
_sz, _sy, _sx = np.meshgrid(np.arange(SUB), np.arange(SUB), np.arange(SUB), indexing="ij")
_OFF_X = ((_sx.ravel() + 0.5) / SUB)
_OFF_Y = ((_sy.ravel() + 0.5) / SUB)
_OFF_Z = ((_sz.ravel() + 0.5) / SUB)
_BITS = (np.uint64(1) << np.arange(SUB ** 3, dtype=np.uint64))


def gas_masks(nx: int, ny: int, nz: int, centres: np.ndarray, diameter) -> np.ndarray:
    """Per-cell 64-bit masks of the sub-cell centres inside the union of the bubbles.

    ``diameter`` is a scalar or one value per bubble.  Cells whose farthest
    corner is strictly inside a sphere are full; cells whose nearest point is
    on or outside it are empty for that sphere; only the cells in between are
    sampled point by point.
    """
    masks = np.zeros((nz, ny, nx), dtype=np.uint64)
    diam = np.broadcast_to(np.asarray(diameter, dtype=np.float64), (len(centres),))
    for (cx, cy, cz), d in zip(centres, diam):
        r = 0.5 * d
        r2 = r * r
        i0, i1 = max(int(np.floor(cx - r)), 0), min(int(np.floor(cx + r)), nx - 1)
        j0, j1 = max(int(np.floor(cy - r)), 0), min(int(np.floor(cy + r)), ny - 1)
        k0, k1 = int(np.floor(cz - r)), int(np.floor(cz + r))
        ii = np.arange(i0, i1 + 1)
        jj = np.arange(j0, j1 + 1)
        kk = np.arange(k0, k1 + 1)            # unwrapped; wrapped when stored
        # Per-axis nearest / farthest squared distances of a cell's extent to the centre.
        def near_far(lo, c):
            a = lo - c
            b = lo + 1.0 - c
            near = np.where((a <= 0.0) & (b >= 0.0), 0.0, np.minimum(a * a, b * b))
            far = np.maximum(a * a, b * b)
            return near, far
        nxd, fxd = near_far(ii.astype(np.float64), cx)
        nyd, fyd = near_far(jj.astype(np.float64), cy)
        nzd, fzd = near_far(kk.astype(np.float64), cz)
        near = nzd[:, None, None] + nyd[None, :, None] + nxd[None, None, :]
        far = fzd[:, None, None] + fyd[None, :, None] + fxd[None, None, :]
        full = far < r2
        part = (~full) & (near < r2)
        kw = np.mod(kk, nz)
        box = masks[np.ix_(kw, jj, ii)]
        box[full] |= _FULL
        if part.any():
            pk, pj, pi = np.nonzero(part)
            px = ii[pi][:, None] + _OFF_X[None, :] - cx
            py = jj[pj][:, None] + _OFF_Y[None, :] - cy
            pz = kk[pk][:, None] + _OFF_Z[None, :] - cz
            inside = (px * px + py * py + pz * pz) < r2
            bits = np.bitwise_or.reduce(np.where(inside, _BITS[None, :], np.uint64(0)), axis=1)
            box[pk, pj, pi] |= bits
        masks[np.ix_(kw, jj, ii)] = box
    return masks


def volume_fraction(nx: int, ny: int, nz: int, centres: np.ndarray, diameter) -> np.ndarray:
    """Gas volume fraction per cell: (sub-cell centres inside any bubble) / 64."""
    masks = gas_masks(nx, ny, nz, centres, diameter)
    return np.bitwise_count(masks).astype(np.float64) / float(SUB ** 3)


def face_velocities(rng: np.random.Generator, nx: int, ny: int, nz: int):
    """Seeded U[-1, 1] face velocities; wall-normal faces are set to zero."""
    shape = (nz, ny, nx)
    u = rng.uniform(-1.0, 1.0, size=shape)
    v = rng.uniform(-1.0, 1.0, size=shape)
    w = rng.uniform(-1.0, 1.0, size=shape)
    u[:, :, nx - 1] = 0.0
    v[:, ny - 1, :] = 0.0
    return u, v, w


def make_case(nx: int, ny: int, nz: int, n_bubbles: int, diameter: float, seed: int,
              min_gap: float = 0.0, name: str = "", velocities: bool = True) -> Case:
    """Bubbles by dart throwing (centre distance >= diameter + min_gap), then face velocities."""
    rng = np.random.default_rng(seed)
    centres = place_bubbles(rng, nx, ny, nz, n_bubbles, diameter, diameter + min_gap)
    alpha = volume_fraction(nx, ny, nz, centres, diameter)
    case = Case(nx, ny, nz, 1.0 / nx, centres, float(diameter), alpha, name=name, seed=seed)
    if velocities:
        case.u, case.v, case.w = face_velocities(rng, nx, ny, nz)
    return case


# Named workloads.  Grid spacing is h = 1/nx, so the duct is [0,1]^2 x [0, nz/nx].
PRESETS = {
    # 32x32x64, 8 bubbles of 8 cells, non-overlapping.
    "duct32": dict(nx=32, ny=32, nz=64, n_bubbles=8, diameter=8.0, seed=1, min_gap=0.0),
    # 128x128x256, 108 bubbles of 16 cells, non-overlapping.
    "duct128": dict(nx=128, ny=128, nz=256, n_bubbles=108, diameter=16.0, seed=2, min_gap=0.0),
    # 256x256x512, 864 bubbles of 13 cells, Poisson-disk with a 2-cell minimum gap.
    "duct256": dict(nx=256, ny=256, nz=512, n_bubbles=864, diameter=13.0, seed=3, min_gap=2.0),
    # 192x192x384, 400 bubbles of 12 cells (first step of the moving sequence).
    "duct192": dict(nx=192, ny=192, nz=384, n_bubbles=400, diameter=12.0, seed=5, min_gap=0.0),
}


def preset(name: str, velocities: bool = True) -> Case:
    p = dict(PRESETS[name])
    return make_case(p.pop("nx"), p.pop("ny"), p.pop("nz"), p.pop("n_bubbles"), p.pop("diameter"),
                     p.pop("seed"), min_gap=p.pop("min_gap"), name=name, velocities=velocities)


def paper_lattice_case(velocities: bool = False) -> Case:
    """The paper's own geometry: 192x192x768 cells, 864 bubbles of 8 cells on a
    regular 6x6x24 array (spacing 32 cells, offset 16)."""
    nx, ny, nz = 192, 192, 768
    centres = lattice_bubbles(nx, ny, nz, (6, 6, 24), (32, 32, 32), (16, 16, 16))
    alpha = volume_fraction(nx, ny, nz, centres, 8.0)
    case = Case(nx, ny, nz, 1.0 / nx, centres, 8.0, alpha, name="paper192x768", seed=6)
    if velocities:
        case.u, case.v, case.w = face_velocities(np.random.default_rng(6), nx, ny, nz)
    return case


def random_small_case(seed: int, nx: int, ny: int, nz: int, n_levels: int = 65):
    """Tiny case with a gas fraction drawn from {0, 1/64, ..., 1} per cell (independent
    of any geometry) plus face velocities; used for brute-force comparisons."""
    rng = np.random.default_rng(seed)
    alpha = rng.integers(0, n_levels, size=(nz, ny, nx)).astype(np.float64) / 64.0
    u, v, w = face_velocities(rng, nx, ny, nz)
    return Case(nx, ny, nz, 1.0 / nx, np.zeros((0, 3)), 0.0, alpha, u, v, w, name="random", seed=seed)


def serving_requests(n_requests: int = 256, rate_hz: float = 40.0, seed: int = 4,
                     grids=((32, 32, 64), (64, 64, 128), (96, 96, 192), (128, 128, 256)),
                     max_void: float = 0.10):
    """Request stream for the serving workload: Poisson arrivals and per-request bubble draws.

    Each request: grid uniform over ``grids``; diameter d ~ U{6..16} clamped to
    nx/2 - 1; count n ~ U{4..200} clamped so that n*pi*d^3/6 <= max_void * N.
    Returns a list of dicts with the arrival time (s), grid, d, n and a per-request seed.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for q in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        g = grids[int(rng.integers(0, len(grids)))]
        d = int(rng.integers(6, 17))
        d = min(d, g[0] // 2 - 1)
        n = int(rng.integers(4, 201))
        cap = int(max_void * g[0] * g[1] * g[2] / (np.pi * d ** 3 / 6.0))
        n = max(1, min(n, cap))
        out.append(dict(index=q, arrival_s=t, grid=g, diameter=float(d), n_bubbles=n,
                        seed=int(rng.integers(0, 2 ** 31 - 1))))
    return out


def moving_sequence(case: Case, steps: int, seed: int = 5, dz: float = 0.5, jitter: float = 0.1):
    """Bubble centres for a time sequence: +dz cells in z per step and a seeded
    U[-jitter, jitter] lateral move, clamped so every bubble stays inside
    [r+1, W-r-1].  Yields ``(step, centres)`` for step = 0 .. steps-1 (step 0 is
    the case's own centres)."""
    rng = np.random.default_rng((seed, 0xB0B))
    c = case.centres.copy()
    r = 0.5 * case.diameter
    for s in range(steps):
        yield s, c.copy()
        c[:, 2] = np.mod(c[:, 2] + dz, case.nz)
        c[:, 0] = np.clip(c[:, 0] + rng.uniform(-jitter, jitter, len(c)), r + 1.0, case.nx - r - 1.0)
        c[:, 1] = np.clip(c[:, 1] + rng.uniform(-jitter, jitter, len(c)), r + 1.0, case.ny - r - 1.0)


def sequence_velocity_perturbation(step: int, nx: int, ny: int, nz: int, seed: int = 5):
    """Seeded U[-1, 1] face-velocity perturbation for one step of the sequence."""
    return face_velocities(np.random.default_rng((seed, step)), nx, ny, nz)
