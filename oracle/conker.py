"""FP64 CPU oracle for the ConKer hot path (mapping, convolution, summation).

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports or calls this
module; only the tests, the smoke check and the CPU-baseline leg of the bench
use it.  It shares no code with the HIP path.

Everything is computed in float64 with NumPy / SciPy, following the paper
(Brown, Mishtaku & Demina, "ConKer: evaluating isotropic correlations of
arbitrary order", arXiv:2108.00015) stage by stage:

* mapping      -- Sec. 2.2 (Input): histograms D and R on a grid of spacing g_s,
                  R normalised to the data total, N = D - R  (Eq. bgsubtracted_map);
* kernels      -- Sec. 2.3 (Kernels): one-cell-thick spherical shells;
* convolution  -- Sec. 2.4 (Convolution): W_i = N *** K_i and B_i = R *** K_i
                  (Eqs. countconv, randconv), done with an FFT as the paper does;
* summation    -- Sec. 2.5: xi_n = sum W_0 W_1 ... W_{n-1} / sum B_0 ... B_{n-1}
                  (Eq. ksin_delta), W_0 = N and B_0 = R.

Readings taken where the paper is silent (each is listed with its reason in the
design notes):

* NGP assignment, half-open cells, index floor((x - origin) / g_s) evaluated in
  float64 from the float32 coordinates; points outside the grid are excluded and
  counted.
* R is normalised with alpha = sum(w_D) / sum(w_R) over in-grid points, and the
  denominator sum B_0...B_{n-1} is evaluated on alpha * R_raw.
* A shell of radius s holds the lattice offsets delta with
  r - 1/2 <= |delta| < r + 1/2, r = s / g_s (cells whose centre lies within half
  a cell of the sphere).
* Convolution is circular on the given grid; bounded surveys are zero-padded so
  that circular equals linear.
* The sum in Eq. ksin_delta runs over every grid cell; the radius tuples are all
  multisets a_1 <= ... <= a_{n-1} of shell indices.
"""
from __future__ import annotations

import itertools
import math
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

WORKERS = max(1, len(os.sched_getaffinity(0)))


# ----------------------------------------------------------------------------
# mapping (Sec. 2.2, Eq. bgsubtracted_map)
# ----------------------------------------------------------------------------

def cell_index(pos: np.ndarray, origin: Sequence[float], cell: float,
               dims: Sequence[int]) -> Tuple[np.ndarray, np.ndarray]:
    """NGP cell of each tracer: floor((x - origin) / g_s) per axis, in float64.

    Returns (int64 [N, 3] cell indices, bool [N] inside-grid mask).
    """
    p = np.asarray(pos, dtype=np.float32).astype(np.float64)
    o = np.asarray(origin, dtype=np.float64)
    c = np.floor((p - o) / np.float64(cell))
    d = np.asarray(dims, dtype=np.float64)
    inside = np.all((c >= 0.0) & (c < d), axis=1)
    c = np.where(inside[:, None], c, 0.0).astype(np.int64)
    return c, inside


def linear_index(c: np.ndarray, dims: Sequence[int]) -> np.ndarray:
    """Row-major (C order, z fastest) linear cell index."""
    ny, nz = int(dims[1]), int(dims[2])
    return (c[:, 0] * ny + c[:, 1]) * nz + c[:, 2]


def histogram(pos: np.ndarray, w: Optional[np.ndarray], origin, cell, dims
              ) -> Tuple[np.ndarray, float, int]:
    """Tracer (or weighted tracer) count per cell, Sec. 2.2.

    Returns (float64 grid of shape dims, sum of in-grid weights, number of
    out-of-grid tracers).
    """
    c, inside = cell_index(pos, origin, cell, dims)
    lin = linear_index(c[inside], dims)
    n_cells = int(np.prod(dims))
    if w is None:
        ww = np.ones(int(inside.sum()), dtype=np.float64)
    else:
        ww = np.asarray(w, dtype=np.float32).astype(np.float64)[inside]
    grid = np.bincount(lin, weights=ww, minlength=n_cells).astype(np.float64)
    return grid.reshape(tuple(int(x) for x in dims)), float(ww.sum()), int((~inside).sum())


def density_deviation(D: np.ndarray, R_raw: np.ndarray, wsum_data: float,
                      wsum_rand: float) -> Tuple[np.ndarray, float]:
    """N = D - R with R = alpha * R_raw normalised to the data total (Eq. bgsubtracted_map).

    Returns (N, alpha)."""
    alpha = wsum_data / wsum_rand
    return D - alpha * R_raw, alpha


# ----------------------------------------------------------------------------
# kernels (Sec. 2.3)
# ----------------------------------------------------------------------------

def shell_reach(r: float) -> int:
    """Largest offset component M that a shell of radius r (cells) can hold."""
    return int(math.ceil(r + 0.5)) - 1


def shell_offsets(r: float) -> np.ndarray:
    """Lattice offsets of the one-cell-thick shell of radius r (in cells).

    S(r) = {delta in Z^3 : (r - 1/2)^2 <= |delta|^2 < (r + 1/2)^2}, compared in
    float64 (exact for the half-integer bounds of integer r).
    """
    if not r >= 0.5:
        raise ValueError("shell radius must be at least half a cell")
    M = shell_reach(r)
    ax = np.arange(-M, M + 1, dtype=np.int64)
    d = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    d2 = (d * d).sum(axis=1).astype(np.float64)
    lo = (r - 0.5) ** 2
    hi = (r + 0.5) ** 2
    return d[(d2 >= lo) & (d2 < hi)]


def check_shell_fits(r: float, dims: Sequence[int]) -> None:
    if 2 * shell_reach(r) + 1 > min(int(x) for x in dims):
        raise ValueError("shell of radius %g cells does not fit the grid %s" % (r, tuple(dims)))


def shell_kernel_grid(r: float, dims: Sequence[int]) -> np.ndarray:
    """Indicator of S(r) laid on the grid with its centre at cell (0,0,0), periodic wrap."""
    check_shell_fits(r, dims)
    k = np.zeros(tuple(int(x) for x in dims), dtype=np.float64)
    d = shell_offsets(r)
    k[d[:, 0] % dims[0], d[:, 1] % dims[1], d[:, 2] % dims[2]] = 1.0
    return k


def shell_spectrum(r: float, dims: Sequence[int]) -> np.ndarray:
    """Full complex DFT of the wrapped shell indicator (unnormalised forward DFT)."""
    return sfft.fftn(shell_kernel_grid(r, dims), workers=WORKERS)


# ----------------------------------------------------------------------------
# convolution (Sec. 2.4, Eqs. countconv, randconv)
# ----------------------------------------------------------------------------

def convolve_shell(F: np.ndarray, r: float, F_hat: Optional[np.ndarray] = None) -> np.ndarray:
    """Map of shell sums C_r(x) = sum_{delta in S(r)} F(x + delta) (circular).

    Computed as the paper does, by FFT: irfft(rfft(F) * rfft(K_r)).  The kernel
    is point-symmetric, so convolution and correlation coincide.
    """
    dims = F.shape
    K = shell_kernel_grid(r, dims)
    if F_hat is None:
        F_hat = sfft.rfftn(F, workers=WORKERS)
    K_hat = sfft.rfftn(K, workers=WORKERS)
    return sfft.irfftn(F_hat * K_hat, s=dims, workers=WORKERS)


def convolve_shells(F: np.ndarray, radii_cells: Sequence[float]) -> np.ndarray:
    """Stack of maps [N_s, nx, ny, nz], one per shell radius (in cells)."""
    F_hat = sfft.rfftn(F, workers=WORKERS)
    return np.stack([convolve_shell(F, r, F_hat) for r in radii_cells])


def direct_shell_sum(F: np.ndarray, r: float, cells: np.ndarray) -> np.ndarray:
    """C_r at the given cells [K, 3] by summing F over the shell offsets directly."""
    dims = np.asarray(F.shape)
    d = shell_offsets(r)
    out = np.empty(len(cells), dtype=np.float64)
    for i, x in enumerate(np.asarray(cells, dtype=np.int64)):
        idx = (x[None, :] + d) % dims[None, :]
        out[i] = F[idx[:, 0], idx[:, 1], idx[:, 2]].sum()
    return out


# ----------------------------------------------------------------------------
# summation (Sec. 2.5, Eqs. ksin_delta, ksi2_delta, ksi3; Sec. 2.6, Eq. ksinDiag)
# ----------------------------------------------------------------------------

def radius_tuples(n_radii: int, n: int) -> List[Tuple[int, ...]]:
    """All multisets a_1 <= ... <= a_{n-1} of shell indices, lexicographic."""
    if n < 2:
        raise ValueError("correlation order must be at least 2")
    return list(itertools.combinations_with_replacement(range(n_radii), n - 1))


def num_tuples(n_radii: int, n: int) -> int:
    return math.comb(n_radii + n - 2, n - 1)


def contract(F: np.ndarray, maps: np.ndarray, n: int,
             tuples: Optional[Iterable[Tuple[int, ...]]] = None,
             chunk: int = 1 << 22) -> np.ndarray:
    """W_n(a_1..a_{n-1}) = sum_x F(x) prod_i C_{a_i}(x) for each radius tuple.

    This is the numerator (F = N, maps W_i) or the denominator (F = R, maps B_i)
    of Eq. ksin_delta, summed over every grid cell; the sum over cells is taken
    in consecutive slices of ``chunk`` cells to bound memory.
    """
    if tuples is None:
        tuples = radius_tuples(maps.shape[0], n)
    tuples = [tuple(t) for t in tuples]
    for t in tuples:
        if len(t) != n - 1:
            raise ValueError("tuple %r does not match order n=%d" % (t, n))
    f = F.reshape(-1)
    C = maps.reshape(maps.shape[0], -1)
    W = np.zeros(len(tuples), dtype=np.float64)
    for s in range(0, f.size, chunk):
        fs = f[s:s + chunk]
        Cs = C[:, s:s + chunk]
        for k, t in enumerate(tuples):
            prod = fs.copy()
            for a in t:
                prod *= Cs[a]
            W[k] += prod.sum()
    return W


def estimator(W_delta: np.ndarray, W_rand_raw: np.ndarray, alpha: float, n: int) -> np.ndarray:
    """xi_n = sum W_0..W_{n-1} / sum B_0..B_{n-1}, with B built on R = alpha R_raw.

    W_rand_raw is the contraction of R_raw; scaling R by alpha scales every
    factor B_i by alpha, so the denominator is alpha^n * W_rand_raw.
    """
    return W_delta / (alpha ** n * W_rand_raw)


def npcf(data_pos, rand_pos, dims, origin, cell, radii, n,
         data_w=None, rand_w=None, tuples=None):
    """End-to-end estimator for one catalog pair: mapping -> convolution -> summation.

    radii are in length units.  Returns a dict with xi, W_delta, W_rand_raw,
    alpha and the intermediate grids.
    """
    D, wd, out_d = histogram(data_pos, data_w, origin, cell, dims)
    R_raw, wr, out_r = histogram(rand_pos, rand_w, origin, cell, dims)
    N, alpha = density_deviation(D, R_raw, wd, wr)
    rc = [float(s) / float(cell) for s in radii]
    maps_N = convolve_shells(N, rc)
    maps_R = convolve_shells(R_raw, rc)
    Wd = contract(N, maps_N, n, tuples)
    Wr = contract(R_raw, maps_R, n, tuples)
    return dict(xi=estimator(Wd, Wr, alpha, n), W_delta=Wd, W_rand_raw=Wr, alpha=alpha,
                N=N, R_raw=R_raw, maps_N=maps_N, maps_R=maps_R,
                wsum_data=wd, wsum_rand=wr, outside=(out_d, out_r))


def diagonal(F: np.ndarray, map_1: np.ndarray, n: int) -> float:
    """Equidistant case, Eq. ksinDiag numerator: sum_x F(x) C_1(x)^(n-1)."""
    return float((F * map_1 ** (n - 1)).sum())


# ----------------------------------------------------------------------------
# continuous tracers (Sec. 2.7, Eqs. densitycont, ksin_cont, ksi2_cont)
# ----------------------------------------------------------------------------

def delta_field(D: np.ndarray, R: np.ndarray) -> np.ndarray:
    """Relative over-density delta = (D - R) / R of two continuous fields on the
    grid (Eq. densitycont).  Cells with R = 0 have no random coverage: they lie
    outside the survey and get delta = 0."""
    D = np.asarray(D, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    out = np.zeros_like(D)
    m = R != 0.0
    out[m] = (D[m] - R[m]) / R[m]
    return out


def npcf_continuous(D: np.ndarray, R: np.ndarray, radii_cells: Sequence[float], n: int,
                    tuples=None) -> np.ndarray:
    """xi_n = sum_x W_0(x) W_1(x; s_1) ... W_{n-1}(x; s_{n-1}) with W_0 = delta and
    W_i = delta *** K_i (Eq. ksin_cont): delta is already normalised, so the sum
    is not divided by anything."""
    delta = delta_field(D, R)
    return contract(delta, convolve_shells(delta, radii_cells), n, tuples)


# ----------------------------------------------------------------------------
# cross-correlation of two tracers (Sec. 2.8)
# ----------------------------------------------------------------------------

def estimator_cross(W_cross: np.ndarray, W_rand_raw: np.ndarray, alpha0: float, alpha1: float,
                    n: int) -> np.ndarray:
    """xi = sum Delta_0 W_1..W_{n-1} / sum B_0 B_1..B_{n-1}, where W_i are the maps of
    tracer 1 and the denominator is built on the common randoms normalised to
    each tracer: B_0 = alpha0 R_raw, B_i = alpha1 (R_raw *** K_i), i.e.
    alpha0 alpha1^(n-1) times the contraction of R_raw."""
    return W_cross / (alpha0 * alpha1 ** (n - 1) * W_rand_raw)


def npcf_cross(data0_pos, data1_pos, rand_pos, dims, origin, cell, radii, n,
               data0_w=None, data1_w=None, rand_w=None, tuples=None):
    """Cross-correlation of tracer 0 (vertex 0) with tracer 1 (the other vertices),
    both background-subtracted against one random catalog.  radii in length units."""
    D0, wd0, _ = histogram(data0_pos, data0_w, origin, cell, dims)
    D1, wd1, _ = histogram(data1_pos, data1_w, origin, cell, dims)
    R_raw, wr, _ = histogram(rand_pos, rand_w, origin, cell, dims)
    N0, a0 = density_deviation(D0, R_raw, wd0, wr)
    N1, a1 = density_deviation(D1, R_raw, wd1, wr)
    rc = [float(s) / float(cell) for s in radii]
    Wc = contract(N0, convolve_shells(N1, rc), n, tuples)
    Wr = contract(R_raw, convolve_shells(R_raw, rc), n, tuples)
    return dict(xi=estimator_cross(Wc, Wr, a0, a1, n), W_cross=Wc, W_rand_raw=Wr, alpha0=a0, alpha1=a1,
                N0=N0, N1=N1, R_raw=R_raw)


# ----------------------------------------------------------------------------
# regions, maps and their distributions (Sec. 3.4, Eq. ksi3combined; Sec. 4.2)
# ----------------------------------------------------------------------------

def combine_regions(W_deltas: Sequence[np.ndarray], W_rands_raw: Sequence[np.ndarray],
                    alphas: Sequence[float], n: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Several regions (e.g. the two galactic caps) combined by adding numerators
    and denominators (Eq. ksi3combined): xi = sum_j W_delta_j / sum_j alpha_j^n W_R_j.
    Returns (xi, numerator, denominator)."""
    num = np.sum([np.asarray(w, dtype=np.float64) for w in W_deltas], axis=0)
    den = np.sum([a ** n * np.asarray(w, dtype=np.float64) for a, w in zip(alphas, W_rands_raw)], axis=0)
    return num / den, num, den


def map_ratio(N: np.ndarray, map_N: np.ndarray, W_rand_raw_2: float, alpha: float) -> np.ndarray:
    """Per-cell W_0 W_1 / <B_0 B_1> for one radius (the maps of Sec. 4.2): N(x) C^N(x)
    over the cell average of B_0 B_1 = alpha^2 R_raw C^R, i.e. alpha^2 W_R2 / N_c.
    Its cell average is the 2pcf of that radius."""
    return N * map_N / (alpha * alpha * W_rand_raw_2 / N.size)


def value_histogram(values: np.ndarray, lo: float, hi: float, n_bins: int) -> np.ndarray:
    """Counts of values in n_bins equal bins of [lo, hi), then one bin of values
    below lo and one of values at or above hi (NaN counts as above)."""
    v = np.asarray(values, dtype=np.float64).ravel()
    counts = np.zeros(n_bins + 2, dtype=np.int64)
    inside = (v >= lo) & (v < hi)
    b = np.floor((v[inside] - lo) / (hi - lo) * n_bins).astype(np.int64)
    b = np.minimum(b, n_bins - 1)
    counts[:n_bins] = np.bincount(b, minlength=n_bins)
    counts[n_bins] = int((v < lo).sum())
    counts[n_bins + 1] = int(v.size - inside.sum() - (v < lo).sum())
    return counts


# ----------------------------------------------------------------------------
# survey front end (Sec. 2.2, Eqs. hubbleint, cartesianx-z, factorizablility)
# ----------------------------------------------------------------------------

def hubble_e(z, Om: float, Ok: float, OL: float):
    """E(z) = sqrt(Om (1+z)^3 + Ok (1+z)^2 + OL), the integrand's denominator of Eq. hubbleint."""
    zp = 1.0 + np.asarray(z, dtype=np.float64)
    return np.sqrt(Om * zp ** 3 + Ok * zp ** 2 + OL)


def comoving_distance(z, Om: float = 0.307, Ok: float = 0.0, OL: float = 0.693,
                      H0: float = 100.0, c: float = 300000.0) -> np.ndarray:
    """r(z) = c/H0 int_0^z dz' / E(z') (Eq. hubbleint), adaptive quadrature per value
    (with H0 = 100 the unit is Mpc/h, as in the paper's runs)."""
    from scipy.integrate import quad
    zz = np.atleast_1d(np.asarray(z, dtype=np.float64))
    out = np.array([quad(lambda t: 1.0 / float(hubble_e(t, Om, Ok, OL)), 0.0, float(v),
                         epsabs=0.0, epsrel=1e-13, limit=200)[0] for v in zz])
    return (c / H0) * out


def sky_to_cartesian(ra_deg, dec_deg, z, **cosmo) -> np.ndarray:
    """Comoving Cartesian positions (Eqs. cartesianx, cartesiany, cartesianz):
    X = r cos(dec) cos(ra), Y = r cos(dec) sin(ra), Z = r sin(dec); float64 [N, 3]."""
    r = comoving_distance(z, **cosmo)
    a = np.radians(np.asarray(ra_deg, dtype=np.float64))
    d = np.radians(np.asarray(dec_deg, dtype=np.float64))
    return np.stack([r * np.cos(d) * np.cos(a), r * np.cos(d) * np.sin(a), r * np.sin(d)], axis=1)


def redshift_of_distance(r, z_max: float, Om: float = 0.307, Ok: float = 0.0, OL: float = 0.693,
                         H0: float = 100.0, c: float = 300000.0, nodes: int = 4001) -> np.ndarray:
    """z(r), the inverse of Eq. hubbleint, by a cubic spline through r(z) evaluated
    with quadrature at `nodes` redshifts of [0, z_max] (r is monotonic in z)."""
    from scipy.interpolate import CubicSpline
    zk = np.linspace(0.0, z_max, nodes)
    rk = comoving_distance(zk, Om, Ok, OL, H0, c)
    return CubicSpline(rk, zk)(np.asarray(r, dtype=np.float64))


def analytic_randoms(dims, origin, cell: float, n_tot: float, p_ang: np.ndarray, ra_range, dec_range,
                     p_z: np.ndarray, z_range, Om: float = 0.307, Ok: float = 0.0, OL: float = 0.693,
                     H0: float = 100.0, c: float = 300000.0) -> np.ndarray:
    """Expected random count per cell for factorizable selection functions
    (Eq. factorizablility): with P_ang a density per steradian on an equal-angle
    (dec, ra) table and P_z a density in z on equal bins, the comoving number
    density is n = N_tot P_ang P_z / (r^2 dr/dz), dr/dz = c / (H0 E(z)), and the
    cell count is n at the cell centre times cell^3.  Cells whose centre falls
    outside the tables get 0."""
    nx, ny, nz = (int(v) for v in dims)
    ix, iy, iz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    X = origin[0] + (ix + 0.5) * cell
    Y = origin[1] + (iy + 0.5) * cell
    Z = origin[2] + (iz + 0.5) * cell
    r = np.sqrt(X * X + Y * Y + Z * Z)
    dec = np.degrees(np.arcsin(Z / r))
    ra = np.degrees(np.arctan2(Y, X)) % 360.0
    # z(r) from a table that reaches past the farthest cell centre (no extrapolation)
    z_hi = max(float(z_range[1]), 0.01)
    while comoving_distance([z_hi], Om, Ok, OL, H0, c)[0] < r.max() and z_hi < 64.0:
        z_hi *= 2.0
    z = redshift_of_distance(r, z_hi, Om, Ok, OL, H0, c)
    nd, na = p_ang.shape
    ia = np.floor((ra - ra_range[0]) / (ra_range[1] - ra_range[0]) * na).astype(np.int64)
    idd = np.floor((dec - dec_range[0]) / (dec_range[1] - dec_range[0]) * nd).astype(np.int64)
    izz = np.floor((z - z_range[0]) / (z_range[1] - z_range[0]) * len(p_z)).astype(np.int64)
    ok = (ia >= 0) & (ia < na) & (idd >= 0) & (idd < nd) & (izz >= 0) & (izz < len(p_z)) & (r > 0)
    out = np.zeros(r.shape)
    drdz = c / (H0 * hubble_e(z, Om, Ok, OL))
    out[ok] = n_tot * p_ang[idd[ok], ia[ok]] * p_z[izz[ok]] / (r[ok] ** 2 * drdz[ok]) * cell ** 3
    return out
