"""Seeded synthetic galaxy-survey stand-ins.

The paper measures on SDSS DR12 CMASS galaxies, their random catalogs and
MultiDark-Patchy mocks (Sec. 3).  None of those data are used here: every
catalog below is drawn from a seeded generator with the shapes of those
workloads (clustered tracers, a larger uniform random catalog filling the same
volume, optional per-object weights).

* Neyman-Scott clustering: a fixed number of parent centres uniform in the
  volume; each offspring picks a parent uniformly and is displaced by an
  isotropic Gaussian of width sigma.  In a bounded volume offspring that fall
  outside are redrawn; in a periodic box they wrap.
* Randoms: uniform in the same volume.
* Weights: log-normal, w = exp(sigma_w * z) with z ~ N(0, 1).

Positions are generated in float64 and handed out as float32 [N, 3]; both the
oracle and the GPU path read the same float32 arrays.  Nothing here computes
any part of the correlation estimator.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Catalog:
    pos: np.ndarray                  # float32 [N, 3]
    w: Optional[np.ndarray] = None   # float32 [N] or None (unit weights)

    def __len__(self) -> int:
        return int(self.pos.shape[0])


@dataclasses.dataclass
class Workload:
    """A grid, a radius bank and the catalogs that fill it."""
    name: str
    dims: tuple                      # (nx, ny, nz)
    origin: tuple                    # lower corner of cell (0, 0, 0)
    cell: float                      # grid spacing g_s
    radii: tuple                     # shell radii in length units
    orders: tuple                    # correlation orders n evaluated
    periodic: bool
    description: str
    make: object = None              # callable(seed_offset=0) -> (data, randoms)

    @property
    def n_cells(self) -> int:
        return int(self.dims[0]) * int(self.dims[1]) * int(self.dims[2])


# ----------------------------------------------------------------------------
# float32 hand-off
# ----------------------------------------------------------------------------

def _to_f32_box(p64: np.ndarray, lo: float, hi: float, periodic: bool) -> np.ndarray:
    """Cast to float32 keeping every point in [lo, hi) per axis.

    A float64 coordinate just below ``hi`` may round up to ``hi`` in float32;
    in a periodic box that point is the same as ``lo`` and is wrapped there.
    Bounded volumes redraw such points before this call.
    """
    p32 = p64.astype(np.float32)
    if periodic:
        hi32, lo32 = np.float32(hi), np.float32(lo)
        p32 = np.where(p32 >= hi32, lo32, p32)
        p32 = np.where(p32 < lo32, lo32, p32)
    return np.ascontiguousarray(p32, dtype=np.float32)


def _inside_box_f32(p64: np.ndarray, lo: float, hi: float) -> np.ndarray:
    p32 = p64.astype(np.float32)
    return np.all((p32 >= np.float32(lo)) & (p32 < np.float32(hi)), axis=1)


# ----------------------------------------------------------------------------
# cubes
# ----------------------------------------------------------------------------

def uniform_box(n: int, lo: float, hi: float, seed: int, periodic: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    p = rng.uniform(lo, hi, size=(n, 3))
    if not periodic:
        bad = ~_inside_box_f32(p, lo, hi)
        while bad.any():
            p[bad] = rng.uniform(lo, hi, size=(int(bad.sum()), 3))
            bad = ~_inside_box_f32(p, lo, hi)
    return _to_f32_box(p, lo, hi, periodic)


def neyman_scott_box(n: int, n_parents: int, sigma: float, lo: float, hi: float,
                     seed: int, periodic: bool = False) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parents = rng.uniform(lo, hi, size=(n_parents, 3))
    which = rng.integers(0, n_parents, size=n)
    p = parents[which] + rng.normal(0.0, sigma, size=(n, 3))
    if periodic:
        p = lo + np.mod(p - lo, hi - lo)
    else:
        bad = ~_inside_box_f32(p, lo, hi)
        while bad.any():
            k = int(bad.sum())
            p[bad] = parents[which[bad]] + rng.normal(0.0, sigma, size=(k, 3))
            bad = ~_inside_box_f32(p, lo, hi)
    return _to_f32_box(p, lo, hi, periodic)


# ----------------------------------------------------------------------------
# sky caps (survey-shaped volumes)
# ----------------------------------------------------------------------------

def _in_cap(p: np.ndarray, r1: float, r2: float, cos_max: float) -> np.ndarray:
    r = np.sqrt((p.astype(np.float32).astype(np.float64) ** 2).sum(axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        c = p[:, 2] / np.where(r > 0, r, 1.0)
    return (r >= r1) & (r < r2) & (c >= cos_max)


def _cap_uniform64(rng, n: int, r1: float, r2: float, half_angle_deg: float) -> np.ndarray:
    cos_max = math.cos(math.radians(half_angle_deg))
    r = np.cbrt(rng.uniform(r1 ** 3, r2 ** 3, size=n))
    ct = rng.uniform(cos_max, 1.0, size=n)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    ph = rng.uniform(0.0, 2.0 * math.pi, size=n)
    return np.stack([r * st * np.cos(ph), r * st * np.sin(ph), r * ct], axis=1)


def uniform_cap(n: int, r1: float, r2: float, half_angle_deg: float, seed: int) -> np.ndarray:
    """Uniform in the spherical shell segment r1 <= r < r2, polar angle <= half_angle."""
    rng = np.random.default_rng(seed)
    cos_max = math.cos(math.radians(half_angle_deg))
    p = _cap_uniform64(rng, n, r1, r2, half_angle_deg)
    bad = ~_in_cap(p, r1, r2, cos_max)
    while bad.any():
        p[bad] = _cap_uniform64(rng, int(bad.sum()), r1, r2, half_angle_deg)
        bad = ~_in_cap(p, r1, r2, cos_max)
    return np.ascontiguousarray(p.astype(np.float32))


def neyman_scott_cap(n: int, n_parents: int, sigma: float, r1: float, r2: float,
                     half_angle_deg: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    cos_max = math.cos(math.radians(half_angle_deg))
    parents = _cap_uniform64(rng, n_parents, r1, r2, half_angle_deg)
    which = rng.integers(0, n_parents, size=n)
    p = parents[which] + rng.normal(0.0, sigma, size=(n, 3))
    bad = ~_in_cap(p, r1, r2, cos_max)
    while bad.any():
        k = int(bad.sum())
        p[bad] = parents[which[bad]] + rng.normal(0.0, sigma, size=(k, 3))
        bad = ~_in_cap(p, r1, r2, cos_max)
    return np.ascontiguousarray(p.astype(np.float32))


def lognormal_weights(n: int, sigma: float, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(n)).astype(np.float32)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def _radii(start: float, stop: float, step: float) -> tuple:
    k = int(round((stop - start) / step))
    return tuple(float(start + i * step) for i in range(k + 1))


def _cube128():
    def make(seed_offset: int = 0, scale: float = 1.0):
        nd = max(1, int(20_000 * scale))
        nr = max(1, int(200_000 * scale))
        d = neyman_scott_box(nd, 400, 10.0, 0.0, 512.0, 101 + seed_offset)
        r = uniform_box(nr, 0.0, 512.0, 102 + seed_offset)
        return Catalog(d), Catalog(r)
    return Workload(
        name="cube512_ns20k_grid128",
        dims=(128, 128, 128), origin=(0.0, 0.0, 0.0), cell=8.0,
        radii=_radii(16.0, 88.0, 8.0), orders=(2, 3), periodic=False,
        description=("20,000 Neyman-Scott points (400 parents, sigma 10) + 200,000 uniform randoms "
                     "in a 512-unit cube; NGP onto 64^3 cells of 8 inside a zero-padded 128^3 grid; "
                     "10 shells 16..88 step 8; unit weights"),
        make=make)


def _cap512():
    # Sky cap along +z: comoving r in [1000, 1900), half-angle 38 degrees so that
    # the cap plus a 34-cell wrap margin fits a 512^3 grid of 5-unit cells.
    r1, r2, ang = 1000.0, 1900.0, 38.0

    def make(seed_offset: int = 0, scale: float = 1.0):
        nd = max(1, int(800_000 * scale))
        nr = 40 * nd
        npar = max(1, int(16_000 * scale))
        d = neyman_scott_cap(nd, npar, 8.0, r1, r2, ang, 201 + seed_offset)
        r = uniform_cap(nr, r1, r2, ang, 202 + seed_offset)
        wd = lognormal_weights(nd, 0.2, 211 + seed_offset)
        wr = lognormal_weights(nr, 0.2, 212 + seed_offset)
        return Catalog(d, wd), Catalog(r, wr)
    return Workload(
        name="cap512_ns800k_r30",
        dims=(512, 512, 512), origin=(-1280.0, -1280.0, 64.0), cell=5.0,
        radii=_radii(20.0, 165.0, 5.0), orders=(2, 3, 4), periodic=False,
        description=("800,000 Neyman-Scott points (16,000 parents, sigma 8) + 32,000,000 uniform "
                     "randoms in a sky cap (axis +z, half-angle 38 deg, r 1000..1900); log-normal "
                     "weights (sigma 0.2) on both; 512^3 grid of 5-unit cells; 30 shells 20..165"),
        make=make)


def _box256():
    L = 1280.0

    def make(seed_offset: int = 0, scale: float = 1.0):
        nd = max(1, int(300_000 * scale))
        nr = 10 * nd
        d = neyman_scott_box(nd, max(1, int(6_000 * scale)), 10.0, 0.0, L, 301 + seed_offset, True)
        r = uniform_box(nr, 0.0, L, 302 + seed_offset, True)
        return Catalog(d), Catalog(r)
    return Workload(
        name="box1280_ns300k_grid256_n5",
        dims=(256, 256, 256), origin=(0.0, 0.0, 0.0), cell=5.0,
        radii=_radii(10.0, 105.0, 5.0), orders=(2, 3, 4, 5), periodic=True,
        description=("300,000 Neyman-Scott points (6,000 parents, sigma 10) + 3,000,000 uniform "
                     "randoms in a periodic 1280-unit box; 256^3 grid of 5-unit cells; 20 shells "
                     "10..105; unit weights"),
        make=make)


def _box1024():
    L = 4096.0

    def make(seed_offset: int = 0, scale: float = 1.0):
        nd = max(1, int(50_000_000 * scale))
        nr = 10 * nd
        d = neyman_scott_box(nd, max(1, int(1_000_000 * scale)), 8.0, 0.0, L, 501 + seed_offset, True)
        r = uniform_box(nr, 0.0, L, 502 + seed_offset, True)
        return Catalog(d), Catalog(r)
    return Workload(
        name="box4096_ns50m_grid1024",
        dims=(1024, 1024, 1024), origin=(0.0, 0.0, 0.0), cell=4.0,
        radii=_radii(8.0, 164.0, 4.0), orders=(3,), periodic=True,
        description=("50M Neyman-Scott points + 500M uniform randoms in a periodic 4096-unit box; "
                     "1024^3 grid of 4-unit cells; 40 shells 8..164"),
        make=make)


WORKLOADS = {w.name: w for w in (_cube128(), _cap512(), _box256(), _box1024())}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def mock_catalog(j: int, grid: int, n: int, scale: float = 1.0, cell: float = 5.0):
    """Mock j of a batch: periodic box of side cell * grid, n Neyman-Scott points
    (n / 50 parents, sigma 10) and 10 n uniform randoms, both times `scale`."""
    L = cell * grid
    nd = max(1, int(n * scale))
    d = neyman_scott_box(nd, max(1, nd // 50), 10.0, 0.0, L, 4000 + 2 * j, True)
    r = uniform_box(10 * nd, 0.0, L, 4001 + 2 * j, True)
    return Catalog(d), Catalog(r)


MOCK_RADII = tuple(float(10 + 5 * i) for i in range(16))   # 10 .. 85, 16 shells


def mock_sizes(n_mocks: int = 64, seed: int = 400) -> Sequence[tuple]:
    """Grid sizes and catalog sizes of a batch of independent periodic mocks."""
    rng = np.random.default_rng(seed)
    g = rng.choice(np.array([96, 128, 192, 256]), size=n_mocks)
    n = rng.integers(50_000, 400_001, size=n_mocks)
    return [(int(a), int(b)) for a, b in zip(g, n)]
