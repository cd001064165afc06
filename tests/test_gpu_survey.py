"""Survey front end through the C ABI against the FP64 oracle: sky coordinates
and redshifts to comoving positions (Eqs. hubbleint, cartesianx-z), and the
expected random count of factorizable selection functions (Eq.
factorizablility).  Bars: positions within 1e-7 of the distance (the float32
rounding of the output); analytic randoms within 1e-8 relative to the largest
cell, on cells farther than 1e-6 of a bin width from every table edge (a cell
centre on an edge may fall on either side within rounding).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(ck):
    c = ck.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cos", [dict(Om=0.307, Ok=0.0, OL=0.693), dict(Om=1.0, Ok=0.0, OL=0.0),
                                 dict(Om=0.3, Ok=0.1, OL=0.6)])
def test_sky_to_cartesian(ck, ctx, cos):
    rng = np.random.default_rng(91)
    n = 3000
    ra = rng.uniform(0, 360, n)
    dec = rng.uniform(-89, 89, n)
    z = rng.uniform(0.0, 2.9, n)
    z[:3] = [0.0, 2.9, 1e-6]
    bad = np.array([-0.1, 3.5, np.nan])
    ra2, dec2, z2 = np.concatenate([ra, [10, 20, 30]]), np.concatenate([dec, [0, 0, 0]]), np.concatenate([z, bad])
    cosmo = ck.Cosmology(omega_m=cos["Om"], omega_k=cos["Ok"], omega_lambda=cos["OL"], z_max=3.0)
    pos = ctx.sky_to_cartesian(*(torch.from_numpy(a).to(DEV) for a in (ra2, dec2, z2)), cosmo=cosmo)
    pos = pos.cpu().numpy().astype(np.float64)
    ref = oc.sky_to_cartesian(ra, dec, z, Om=cos["Om"], Ok=cos["Ok"], OL=cos["OL"])
    r = np.linalg.norm(ref, axis=1)
    err = np.abs(pos[:n] - ref).max(axis=1)
    assert np.all(err <= 1e-7 * np.maximum(r, 1.0)), float((err / np.maximum(r, 1.0)).max())
    assert np.all(np.isnan(pos[n:]))
    # distances at the paper's redshift range are positive and increasing
    order = np.argsort(z)
    assert np.all(np.diff(np.linalg.norm(pos[:n][order], axis=1)) >= -1e-3)


def test_analytic_randoms(ck, ctx):
    rng = np.random.default_rng(92)
    p_ang = rng.uniform(0.5, 1.5, size=(18, 36)) / (4 * math.pi)
    p_z = rng.uniform(0.5, 1.5, size=5) / 0.1
    z_range, ra_range, dec_range = (0.1, 0.2), (0.0, 360.0), (-90.0, 90.0)
    dims, cell = (128, 128, 128), 10.0
    origin = (-640.0, -640.0, -640.0)
    grid = ck.Grid(dims, origin, cell)
    cosmo = ck.Cosmology(z_max=0.5)
    R = ctx.analytic_randoms(grid, 1e6, torch.from_numpy(p_ang).to(DEV), ra_range, dec_range,
                             torch.from_numpy(p_z).to(DEV), z_range, cosmo=cosmo).cpu().numpy()
    ref = oc.analytic_randoms(dims, origin, cell, 1e6, p_ang, ra_range, dec_range, p_z, z_range)
    # cells away from every table edge
    ix, iy, iz = np.meshgrid(*(np.arange(d) for d in dims), indexing="ij")
    X, Y, Z = (origin[k] + (g + 0.5) * cell for k, g in enumerate((ix, iy, iz)))
    r = np.sqrt(X * X + Y * Y + Z * Z)
    zz = oc.redshift_of_distance(r, 0.5)
    dec = np.degrees(np.arcsin(Z / r))
    ra = np.degrees(np.arctan2(Y, X)) % 360.0

    def far(v, lo, hi, nb):
        t = (v - lo) / (hi - lo) * nb
        return np.abs(t - np.round(t)) > 1e-6

    keep = far(zz, *z_range, len(p_z)) & far(ra, *ra_range, 36) & far(dec, *dec_range, 18)
    assert keep.mean() > 0.99
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(R[keep] - ref[keep]).max() <= 1e-8 * scale
    assert abs(R.sum() - ref.sum()) <= 1e-3 * ref.sum()


def test_front_end_errors(ck, ctx):
    t = torch.zeros(4, dtype=torch.float64, device=DEV)
    with pytest.raises(ck.ConkerError):
        ctx.sky_to_cartesian(t, t, t, cosmo=ck.Cosmology(z_max=0.0))
    with pytest.raises(ck.ConkerError):   # E(z)^2 < 0 somewhere in [0, z_max]
        ctx.sky_to_cartesian(t, t, t, cosmo=ck.Cosmology(omega_m=0.0, omega_k=-2.0, omega_lambda=1.0))
    grid = ck.Grid((32, 32, 32), (0, 0, 0), 1.0)
    pa = torch.ones((2, 2), dtype=torch.float64, device=DEV)
    pz = torch.ones(2, dtype=torch.float64, device=DEV)
    with pytest.raises(ck.ConkerError):   # redshift table beyond z_max
        ctx.analytic_randoms(grid, 1.0, pa, (0, 360), (-90, 90), pz, (0.1, 4.0), cosmo=ck.Cosmology(z_max=3.0))
