"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the piece of mathematics) it checks.
All run on the CPU in seconds.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import brute
from oracle import conker as oc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers: tiny clustered catalogs on a zero-padded grid
# ---------------------------------------------------------------------------

def _tiny_catalog(n_data, n_rand, box, seed, weighted=False):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, box, size=(3, 3))
    d = centres[rng.integers(0, 3, n_data)] + rng.normal(0, box / 8, size=(n_data, 3))
    d = np.clip(d, 0, box - 1e-3).astype(np.float32)
    r = rng.uniform(0, box, size=(n_rand, 3)).astype(np.float32)
    wd = rng.uniform(0.5, 1.5, n_data).astype(np.float32) if weighted else None
    wr = rng.uniform(0.5, 1.5, n_rand).astype(np.float32) if weighted else None
    return d, r, wd, wr


def _theta_r3(t_max):
    """r_3(t) = #{(x,y,z) in Z^3 : x^2+y^2+z^2 = t}, from the cube of the theta series."""
    theta = np.zeros(t_max + 1, dtype=np.int64)
    k = 0
    while k * k <= t_max:
        theta[k * k] += 1 if k == 0 else 2
        k += 1
    two = np.convolve(theta, theta)[: t_max + 1]
    return np.convolve(two, theta)[: t_max + 1]


# ---------------------------------------------------------------------------
# P1, P2 -- mapping (Sec. 2.2, Eq. bgsubtracted_map)
# ---------------------------------------------------------------------------

def test_histogram_counts_match_dictionary_count():
    """P1: unit weights give integer tracer counts per cell; out-of-grid tracers excluded."""
    rng = np.random.default_rng(1)
    pos = rng.uniform(-3.0, 35.0, size=(5000, 3)).astype(np.float32)
    dims, origin, cell = (8, 9, 10), (0.0, 0.5, -1.0), 3.5
    grid, wsum, outside = oc.histogram(pos, None, origin, cell, dims)
    counts = {}
    n_out = 0
    for p in pos:
        c = tuple(int(math.floor((float(p[k]) - origin[k]) / cell)) for k in range(3))
        if all(0 <= c[k] < dims[k] for k in range(3)):
            counts[c] = counts.get(c, 0) + 1
        else:
            n_out += 1
    ref = np.zeros(dims)
    for c, v in counts.items():
        ref[c] = v
    assert np.array_equal(grid, ref)
    assert outside == n_out
    assert wsum == len(pos) - n_out


def test_histogram_weighted_total():
    """P1: the weighted histogram sums to the in-grid weight total."""
    rng = np.random.default_rng(2)
    pos = rng.uniform(0, 20, size=(3000, 3)).astype(np.float32)
    w = rng.lognormal(0, 0.2, 3000).astype(np.float32)
    grid, wsum, outside = oc.histogram(pos, w, (0, 0, 0), 2.0, (10, 10, 10))
    assert outside == 0
    assert math.isclose(grid.sum(), float(w.astype(np.float64).sum()), rel_tol=1e-13)
    assert math.isclose(wsum, grid.sum(), rel_tol=1e-13)


def test_density_deviation_sums_to_zero():
    """P2: N = D - alpha R with alpha = sum w_D / sum w_R has zero total."""
    d, r, wd, wr = _tiny_catalog(500, 5000, 16.0, 3, weighted=True)
    D, sd, _ = oc.histogram(d, wd, (0, 0, 0), 1.0, (16, 16, 16))
    R, sr, _ = oc.histogram(r, wr, (0, 0, 0), 1.0, (16, 16, 16))
    N, alpha = oc.density_deviation(D, R, sd, sr)
    assert abs(N.sum()) < 1e-10 * D.sum()
    assert math.isclose(alpha, sd / sr)


# ---------------------------------------------------------------------------
# P3 -- shell kernels (Sec. 2.3)
# ---------------------------------------------------------------------------

def test_r3_theta_series_textbook_values():
    """The theta-series counter reproduces r_3(t) for t = 0..12 (sums of three squares)."""
    assert list(_theta_r3(12)) == [1, 6, 12, 8, 6, 24, 24, 0, 12, 30, 24, 24, 8]


@pytest.mark.parametrize("m", list(range(1, 42)))
def test_shell_size_equals_theta_series(m):
    """P3: |S_m| = sum of r_3(t) over m^2 - m + 1 <= t <= m^2 + m (one-cell-thick shell)."""
    r3 = _theta_r3(m * m + m)
    expect = int(r3[m * m - m + 1: m * m + m + 1].sum())
    assert len(oc.shell_offsets(float(m))) == expect


def test_shell_sizes_small_and_asymptotic():
    sizes = [len(oc.shell_offsets(float(m))) for m in range(1, 12)]
    assert sizes[:3] == [18, 62, 98]
    for m in (10, 20, 30, 40):
        n = len(oc.shell_offsets(float(m)))
        assert abs(n / (4 * math.pi * m * m) - 1) < 0.06


def test_shells_partition_lattice_and_are_cubic_symmetric():
    """P3: shells m = 1..6 partition the nonzero offsets with |d| < 6.5, each invariant under
    the 48 signed axis permutations."""
    seen = set()
    for m in range(1, 7):
        s = {tuple(int(v) for v in d) for d in oc.shell_offsets(float(m))}
        assert not (s & seen)
        seen |= s
        for perm in itertools.permutations(range(3)):
            for signs in itertools.product((1, -1), repeat=3):
                t = {tuple(signs[k] * d[perm[k]] for k in range(3)) for d in s}
                assert t == s
    box = [(x, y, z) for x in range(-6, 7) for y in range(-6, 7) for z in range(-6, 7)
           if 0 < x * x + y * y + z * z < 6.5 ** 2]
    assert seen == set(box)


def test_shell_noninteger_radius_half_open():
    """Reading of non-integer radii: the same half-open rule with real r."""
    s = oc.shell_offsets(11.46)
    d = np.sqrt((s.astype(float) ** 2).sum(1))
    assert d.min() >= 10.96 - 1e-12 and d.max() < 11.96


def test_shell_spectrum_real_even_and_dc():
    """P3: the wrapped shell is point-symmetric, so its DFT is real; the DC term is |S|."""
    dims = (16, 18, 20)
    for r in (1.0, 3.0, 4.5):
        K = oc.shell_spectrum(r, dims)
        assert np.abs(K.imag).max() < 1e-10
        assert math.isclose(K[0, 0, 0].real, len(oc.shell_offsets(r)), rel_tol=1e-14)


def test_shell_must_fit_grid():
    with pytest.raises(ValueError):
        oc.shell_kernel_grid(8.0, (16, 16, 16))
    with pytest.raises(ValueError):
        oc.shell_offsets(0.4)


# ---------------------------------------------------------------------------
# P4 -- convolution maps (Sec. 2.4)
# ---------------------------------------------------------------------------

def test_maps_equal_direct_shell_sums_integer_field():
    """P4: FFT maps equal the real-space shell sums of an integer field at every cell."""
    rng = np.random.default_rng(4)
    F = rng.integers(-3, 4, size=(12, 14, 16)).astype(np.float64)
    cells = np.array(list(itertools.product(range(12), range(14), range(16))))
    for r in (1.0, 2.0, 3.0, 5.0):
        fft_map = oc.convolve_shell(F, r)
        direct = oc.direct_shell_sum(F, r, cells).reshape(F.shape)
        assert np.abs(fft_map - direct).max() < 1e-9


def test_map_total_and_linearity():
    """P4: sum_x C_m = |S_m| sum_x F; the map is linear in F."""
    rng = np.random.default_rng(5)
    F = rng.normal(size=(16, 16, 16))
    G = rng.normal(size=(16, 16, 16))
    for r in (2.0, 4.0):
        C = oc.convolve_shell(F, r)
        assert math.isclose(C.sum(), len(oc.shell_offsets(r)) * F.sum(), rel_tol=1e-9, abs_tol=1e-9)
        lin = oc.convolve_shell(2.0 * F - 3.0 * G, r)
        assert np.allclose(lin, 2.0 * C - 3.0 * oc.convolve_shell(G, r), atol=1e-10)


# ---------------------------------------------------------------------------
# P5 -- brute force over tracer tuples (Eq. ksin_delta)
# ---------------------------------------------------------------------------

def _grid_setup():
    return (16, 16, 16), (0.0, 0.0, 0.0), 1.0


@pytest.mark.parametrize("n,shells,n_data,n_rand", [
    (2, [(1,), (2,), (3,)], 12, 24),
    (3, [(1, 1), (1, 3), (2, 3)], 10, 20),
    (4, [(1, 1, 2), (1, 2, 3)], 6, 10),
    (5, [(1, 1, 2, 3)], 4, 7),
])
def test_oracle_matches_explicit_tuple_enumeration(n, shells, n_data, n_rand):
    """P5: W^Delta_n and W^R_n from grid + FFT maps + contraction equal the explicit sum
    over tracer tuples, with data weights +w and random weights -alpha w."""
    dims, origin, cell = _grid_setup()
    d, r, wd, wr = _tiny_catalog(n_data, n_rand, 8.0, 10 + n, weighted=True)
    res = oc.npcf(d, r, dims, origin, cell, [1.0, 2.0, 3.0], n, wd, wr, tuples=[tuple(a - 1 for a in s) for s in shells])
    cells, u, alpha, cr, wrr = brute.signed_tracers(d, r, origin, cell, dims, wd, wr)
    assert math.isclose(alpha, res["alpha"], rel_tol=1e-14)
    for k, s in enumerate(shells):
        ref_d = brute.tuple_sum(cells, u, s, dims, periodic=False)
        ref_r = brute.tuple_sum(cr, wrr, s, dims, periodic=False)
        assert math.isclose(res["W_delta"][k], ref_d, rel_tol=1e-9, abs_tol=1e-9)
        assert math.isclose(res["W_rand_raw"][k], ref_r, rel_tol=1e-9, abs_tol=1e-9)


@pytest.mark.parametrize("periodic", [False, True])
def test_oracle_matches_pair_factorised_sum_all_tuples(periodic):
    """P5 at a larger size: every tuple of n = 2..5 against the tracer-pair sum."""
    dims, origin, cell = (20, 20, 20), (0.0, 0.0, 0.0), 1.0
    box = 10.0 if not periodic else 20.0
    d, r, wd, wr = _tiny_catalog(120, 240, box, 77, weighted=True)
    radii = [1.0, 2.0, 3.0, 4.0]
    cells, u, alpha, cr, wrr = brute.signed_tracers(d, r, origin, cell, dims, wd, wr)
    for n in (2, 3, 4, 5):
        res = oc.npcf(d, r, dims, origin, cell, radii, n, wd, wr)
        for k, t in enumerate(oc.radius_tuples(len(radii), n)):
            s = [a + 1 for a in t]
            ref_d = brute.pair_factorised_sum(cells, u, s, dims, periodic)
            ref_r = brute.pair_factorised_sum(cr, wrr, s, dims, periodic)
            assert math.isclose(res["W_delta"][k], ref_d, rel_tol=1e-9, abs_tol=1e-8), (n, t)
            assert math.isclose(res["W_rand_raw"][k], ref_r, rel_tol=1e-9, abs_tol=1e-8), (n, t)


# ---------------------------------------------------------------------------
# P6, P12 -- symmetry and the diagonal (Eq. ksinDiag)
# ---------------------------------------------------------------------------

def test_permutation_symmetry_and_diagonal():
    rng = np.random.default_rng(6)
    F = rng.normal(size=(16, 16, 16))
    radii = [1.0, 2.0, 3.5]
    maps = oc.convolve_shells(F, radii)
    for n in (3, 4, 5):
        full = list(itertools.product(range(3), repeat=n - 1))
        W = oc.contract(F, maps, n, full)
        lookup = dict(zip(full, W))
        for t, v in lookup.items():
            assert math.isclose(v, lookup[tuple(sorted(t))], rel_tol=1e-12, abs_tol=1e-12)
        for m in range(3):
            assert math.isclose(lookup[(m,) * (n - 1)], oc.diagonal(F, maps[m], n), rel_tol=1e-12)


# ---------------------------------------------------------------------------
# P7 -- n = 2 identities
# ---------------------------------------------------------------------------

def test_n2_equals_autocorrelation_and_parseval():
    rng = np.random.default_rng(7)
    dims = (16, 12, 10)
    F = rng.normal(size=dims)
    Fh = np.fft.fftn(F)
    auto = np.fft.ifftn(np.abs(Fh) ** 2).real    # A(d) = sum_x F(x) F(x + d)
    radii = [1.0, 2.0, 3.0, 4.0]
    W2 = oc.contract(F, oc.convolve_shells(F, radii), 2)
    for k, r in enumerate(radii):
        d = oc.shell_offsets(r)
        via_auto = auto[d[:, 0] % dims[0], d[:, 1] % dims[1], d[:, 2] % dims[2]].sum()
        Kh = oc.shell_spectrum(r, dims).real
        parseval = (np.abs(Fh) ** 2 * Kh).sum() / F.size
        assert math.isclose(W2[k], via_auto, rel_tol=1e-10)
        assert math.isclose(W2[k], parseval, rel_tol=1e-10)


# ---------------------------------------------------------------------------
# P8, P9 -- closed forms
# ---------------------------------------------------------------------------

def test_uniform_field_closed_form():
    """P8: F = rho everywhere on a periodic grid -> W_n = N_c rho^n prod |S_a|."""
    dims = (12, 12, 12)
    rho = 1.75
    F = np.full(dims, rho)
    radii = [1.0, 2.0, 3.0]
    sizes = [len(oc.shell_offsets(r)) for r in radii]
    maps = oc.convolve_shells(F, radii)
    for n in (2, 3, 4, 5):
        W = oc.contract(F, maps, n)
        for k, t in enumerate(oc.radius_tuples(3, n)):
            ref = F.size * rho ** n * np.prod([sizes[a] for a in t])
            assert math.isclose(W[k], ref, rel_tol=1e-11)


def test_two_points_closed_form():
    """P9: two unit tracers at lattice separation d: W_2(m) = 2[m = round|d|],
    W_3(a, b) = 2[a = b = round|d|] (degenerate vertices kept, as the estimator is written)."""
    dims = (20, 20, 20)
    F = np.zeros(dims)
    F[3, 4, 5] = 1.0
    F[3 + 2, 4 + 1, 5 + 2] = 1.0   # |d| = 3
    radii = [1.0, 2.0, 3.0, 4.0]
    maps = oc.convolve_shells(F, radii)
    W2 = oc.contract(F, maps, 2)
    assert np.allclose(W2, [0, 0, 2, 0], atol=1e-12)
    W3 = oc.contract(F, maps, 3)
    for k, (a, b) in enumerate(oc.radius_tuples(4, 3)):
        assert abs(W3[k] - (2.0 if a == b == 2 else 0.0)) < 1e-12


# ---------------------------------------------------------------------------
# P10 -- equivariance; P13 -- region additivity (Eq. ksi3combined)
# ---------------------------------------------------------------------------

def test_translation_and_cubic_group_invariance():
    rng = np.random.default_rng(8)
    F = rng.normal(size=(16, 16, 16))
    radii = [1.0, 2.0, 3.0]
    ref = oc.contract(F, oc.convolve_shells(F, radii), 3)
    G = np.roll(F, shift=(3, -5, 7), axis=(0, 1, 2))
    assert np.allclose(oc.contract(G, oc.convolve_shells(G, radii), 3), ref, rtol=1e-10)
    H = np.flip(np.transpose(F, (2, 0, 1)), axis=1)
    assert np.allclose(oc.contract(H, oc.convolve_shells(H, radii), 3), ref, rtol=1e-10)


def test_weight_scaling():
    """P10: scaling every weight by c multiplies both parts by c^n; xi is unchanged."""
    dims, origin, cell = (16, 16, 16), (0.0, 0.0, 0.0), 1.0
    d, r, wd, wr = _tiny_catalog(200, 800, 8.0, 9, weighted=True)
    a = oc.npcf(d, r, dims, origin, cell, [1.0, 2.0], 3, wd, wr)
    c = 2.0
    b = oc.npcf(d, r, dims, origin, cell, [1.0, 2.0], 3, wd * np.float32(c), wr * np.float32(c))
    assert np.allclose(b["W_delta"], c ** 3 * a["W_delta"], rtol=1e-10)
    assert np.allclose(b["W_rand_raw"], c ** 3 * a["W_rand_raw"], rtol=1e-10)
    assert np.allclose(b["xi"], a["xi"], rtol=1e-10)


def test_region_additivity():
    """P13: two fields in sub-boxes further apart than the largest shell: numerators add."""
    rng = np.random.default_rng(10)
    dims = (32, 16, 16)
    F1 = np.zeros(dims)
    F2 = np.zeros(dims)
    F1[2:8, 2:8, 2:8] = rng.normal(size=(6, 6, 6))
    F2[18:24, 2:8, 2:8] = rng.normal(size=(6, 6, 6))
    radii = [1.0, 2.0, 3.0]
    for n in (2, 3, 4):
        W = oc.contract(F1 + F2, oc.convolve_shells(F1 + F2, radii), n)
        W1 = oc.contract(F1, oc.convolve_shells(F1, radii), n)
        W2 = oc.contract(F2, oc.convolve_shells(F2, radii), n)
        assert np.allclose(W, W1 + W2, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------------------------
# P11 -- distance calibration (Sec. 3.1): RMS of the true separation ~ g_s / 2
# ---------------------------------------------------------------------------

def test_distance_calibration_rms_matches_paper():
    """P11: for tracer pairs whose NGP cells lie on the shell of a 60-unit kernel at g_s = 5,
    the true separation has an RMS spread of about half a cell (the paper's 2.5)."""
    with open(os.path.join(GOLDEN, "calibration_rms.json")) as fh:
        gold = json.load(fh)
    g, s = gold["cell"], gold["radius"]
    m = s / g
    rng = np.random.default_rng(11)
    n = 400_000
    # random pairs: first tracer uniform in a cell-aligned box, second at a random
    # offset of length near s (uniform in a thick spherical shell around the first)
    a = rng.uniform(0, 50 * g, size=(n, 3))
    rad = np.cbrt(rng.uniform((s - 2 * g) ** 3, (s + 2 * g) ** 3, size=n))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    b = a + rad[:, None] * v
    ca = np.floor(a / g).astype(np.int64)
    cb = np.floor(b / g).astype(np.int64)
    shell = {tuple(int(x) for x in d) for d in oc.shell_offsets(m)}
    on = np.array([tuple(x) in shell for x in (cb - ca)])
    true = rad[on]
    rms = float(np.sqrt(((true - true.mean()) ** 2).mean()))
    assert abs(rms - gold["rms"]) < gold["tolerance"], rms
    assert abs(true.mean() - s) < 0.5


# ---------------------------------------------------------------------------
# continuous delta fields (Sec. 2.7) and cross-correlation (Sec. 2.8)
# ---------------------------------------------------------------------------

def test_delta_field_closed_forms():
    rng = np.random.default_rng(30)
    R = rng.uniform(0.5, 2.0, size=(8, 8, 8))
    R[0] = 0.0                                   # no random coverage
    assert np.all(oc.delta_field(2.0 * R, R)[1:] == 1.0)
    assert np.all(oc.delta_field(R, R) == 0.0)
    D = rng.uniform(0.0, 3.0, size=R.shape)
    d = oc.delta_field(D, R)
    assert np.all(d[0] == 0.0)
    assert np.allclose(d[1:] * R[1:] + R[1:], D[1:], rtol=1e-14, atol=0)


def test_continuous_uniform_delta_closed_form():
    """delta = c on every cell of a periodic grid -> xi_n = N_c c^n prod |S_a| (Eq. ksin_cont)."""
    dims = (12, 12, 12)
    R = np.full(dims, 1.5)
    c = -0.3
    D = (1.0 + c) * R
    radii = [1.0, 2.0, 2.5]
    sizes = [len(oc.shell_offsets(r)) for r in radii]
    for n in (2, 3, 4):
        xi = oc.npcf_continuous(D, R, radii, n)
        for k, t in enumerate(oc.radius_tuples(len(radii), n)):
            ref = np.prod(dims) * (D[0, 0, 0] / R[0, 0, 0] - 1.0) ** n * np.prod([sizes[a] for a in t])
            assert math.isclose(xi[k], ref, rel_tol=1e-10)


def test_cross_of_a_tracer_with_itself_is_the_auto_estimator():
    dims, origin, cell = _grid_setup()
    d, r, wd, wr = _tiny_catalog(40, 200, 12.0, 31, weighted=True)
    for n in (2, 3):
        auto = oc.npcf(d, r, dims, origin, cell, [1.0, 2.0, 3.0], n, wd, wr)
        cross = oc.npcf_cross(d, d, r, dims, origin, cell, [1.0, 2.0, 3.0], n, wd, wd, wr)
        assert np.allclose(cross["W_cross"], auto["W_delta"], rtol=1e-12, atol=1e-12)
        assert np.allclose(cross["xi"], auto["xi"], rtol=1e-12, atol=1e-12)


def test_cross_matches_explicit_tracer_sums_and_n2_symmetry():
    """Cross W_n against the two-set tracer sum (vertex 0 from tracer 0 and its
    randoms, the others from tracer 1 and its randoms); W_2 is symmetric in the
    two tracers."""
    dims, origin, cell = (20, 20, 20), (0.0, 0.0, 0.0), 1.0
    d0, r, w0, wr = _tiny_catalog(60, 240, 10.0, 32, weighted=True)
    d1, _, w1, _ = _tiny_catalog(50, 10, 10.0, 33, weighted=True)
    radii = [1.0, 2.0, 3.0]
    c0, u0, a0, cr, wrr = brute.signed_tracers(d0, r, origin, cell, dims, w0, wr)
    c1, u1, a1, _, _ = brute.signed_tracers(d1, r, origin, cell, dims, w1, wr)
    for n in (2, 3, 4):
        res = oc.npcf_cross(d0, d1, r, dims, origin, cell, radii, n, w0, w1, wr)
        assert math.isclose(res["alpha0"], a0, rel_tol=1e-14) and math.isclose(res["alpha1"], a1, rel_tol=1e-14)
        for k, t in enumerate(oc.radius_tuples(len(radii), n)):
            ref = brute.cross_tuple_sum(c0, u0, c1, u1, [a + 1 for a in t], dims, False)
            assert math.isclose(res["W_cross"][k], ref, rel_tol=1e-9, abs_tol=1e-8), (n, t)
    w01 = oc.npcf_cross(d0, d1, r, dims, origin, cell, radii, 2, w0, w1, wr)["W_cross"]
    w10 = oc.npcf_cross(d1, d0, r, dims, origin, cell, radii, 2, w1, w0, wr)["W_cross"]
    assert np.allclose(w01, w10, rtol=1e-10, atol=1e-9)


# ---------------------------------------------------------------------------
# regions combined (Eq. ksi3combined), maps of W_0 W_1 / <B_0 B_1>, histograms
# ---------------------------------------------------------------------------

def test_combined_regions_equal_the_union_estimator():
    """Two regions far apart with equal alpha: combining their numerators and
    denominators gives the estimator of the union catalog."""
    dims, origin, cell = (40, 16, 16), (0.0, 0.0, 0.0), 1.0
    rng = np.random.default_rng(40)
    d1 = rng.uniform(1, 8, size=(60, 3)).astype(np.float32)
    r1 = rng.uniform(1, 8, size=(300, 3)).astype(np.float32)
    d2 = (rng.uniform(1, 8, size=(60, 3)) + [24, 0, 0]).astype(np.float32)
    r2 = (rng.uniform(1, 8, size=(300, 3)) + [24, 0, 0]).astype(np.float32)
    radii = [1.0, 2.0, 3.0]
    for n in (2, 3):
        a = oc.npcf(d1, r1, dims, origin, cell, radii, n)
        b = oc.npcf(d2, r2, dims, origin, cell, radii, n)
        u = oc.npcf(np.concatenate([d1, d2]), np.concatenate([r1, r2]), dims, origin, cell, radii, n)
        assert a["alpha"] == b["alpha"] == u["alpha"]
        xi, num, den = oc.combine_regions([a["W_delta"], b["W_delta"]], [a["W_rand_raw"], b["W_rand_raw"]],
                                          [a["alpha"], b["alpha"]], n)
        assert np.allclose(xi, u["xi"], rtol=1e-12, atol=0)
        single = oc.combine_regions([a["W_delta"]], [a["W_rand_raw"]], [a["alpha"]], n)[0]
        assert np.allclose(single, a["xi"], rtol=1e-14, atol=0)


def test_map_ratio_average_is_the_2pcf():
    dims, origin, cell = (16, 16, 16), (0.0, 0.0, 0.0), 1.0
    d, r, wd, wr = _tiny_catalog(200, 2000, 16.0, 41, weighted=True)
    res = oc.npcf(d, r, dims, origin, cell, [2.0, 3.0, 5.0], 2, wd, wr)
    for m in range(3):
        mp = oc.map_ratio(res["N"], res["maps_N"][m], res["W_rand_raw"][m], res["alpha"])
        assert math.isclose(mp.mean(), res["xi"][m], rel_tol=1e-12)


def test_value_histogram_edges():
    v = np.array([-1.0, 0.0, 0.25, 0.5, 0.999, 1.0, 2.0, np.nan])
    c = oc.value_histogram(v, 0.0, 1.0, 4)
    assert c.tolist() == [1, 1, 1, 1, 1, 3]   # [0,.25) [.25,.5) [.5,.75) [.75,1) below above
    rng = np.random.default_rng(42)
    w = rng.normal(size=10000)
    c = oc.value_histogram(w, -2.0, 2.0, 16)
    ref, _ = np.histogram(w[(w >= -2) & (w < 2)], bins=16, range=(-2.0, 2.0))
    assert np.array_equal(c[:16], ref) and c[16] == (w < -2).sum() and c[17] == (w >= 2).sum()


# ---------------------------------------------------------------------------
# survey front end (Eqs. hubbleint, cartesian, factorizablility)
# ---------------------------------------------------------------------------

def test_comoving_distance_closed_forms():
    z = np.array([0.0, 0.1, 0.57, 1.0, 2.5])
    c, H0 = 300000.0, 100.0
    eds = oc.comoving_distance(z, Om=1.0, Ok=0.0, OL=0.0)       # Einstein-de Sitter
    assert np.allclose(eds, 2 * c / H0 * (1 - 1 / np.sqrt(1 + z)), rtol=1e-12, atol=1e-9)
    lam = oc.comoving_distance(z, Om=0.0, Ok=0.0, OL=1.0)       # de Sitter
    assert np.allclose(lam, c / H0 * z, rtol=1e-12, atol=1e-9)
    cur = oc.comoving_distance(z, Om=0.0, Ok=1.0, OL=0.0)       # empty, E = 1 + z
    assert np.allclose(cur, c / H0 * np.log1p(z), rtol=1e-12, atol=1e-9)
    # the paper's cosmology at the CMASS median redshift: ~1.5 Gpc/h
    assert 1400.0 < oc.comoving_distance([0.57])[0] < 1600.0


def test_sky_to_cartesian_geometry_and_inverse():
    rng = np.random.default_rng(90)
    ra, dec, z = rng.uniform(0, 360, 50), rng.uniform(-80, 80, 50), rng.uniform(0.2, 0.8, 50)
    xyz = oc.sky_to_cartesian(ra, dec, z)
    r = np.linalg.norm(xyz, axis=1)
    assert np.allclose(r, oc.comoving_distance(z), rtol=1e-13)
    assert np.allclose(np.degrees(np.arcsin(xyz[:, 2] / r)), dec, atol=1e-9)
    assert np.allclose(np.degrees(np.arctan2(xyz[:, 1], xyz[:, 0])) % 360.0, ra, atol=1e-9)
    # z(r) inverts r(z); Einstein-de Sitter inverse in closed form
    assert np.allclose(oc.redshift_of_distance(r, 1.0), z, atol=1e-10)
    ze = oc.redshift_of_distance(np.array([500.0, 1500.0, 3000.0]), 3.0, Om=1.0, Ok=0.0, OL=0.0)
    rr = np.array([500.0, 1500.0, 3000.0]) * 100.0 / (2 * 300000.0)
    assert np.allclose(ze, 1 / (1 - rr) ** 2 - 1, atol=1e-10)


def test_analytic_randoms_integrate_to_n_tot():
    """A full-sky, constant-P_z shell sampled on a fine grid holds about N_tot
    expected randoms (midpoint rule), and nothing outside the z range."""
    p_ang = np.full((18, 36), 1.0 / (4 * np.pi))         # uniform per steradian
    z_range = (0.1, 0.2)
    p_z = np.full(4, 1.0 / (z_range[1] - z_range[0]))
    r0, r1 = oc.comoving_distance(list(z_range))
    g = 8.0
    nside = int(np.ceil(2 * r1 / g)) + 2
    nside += nside % 2
    origin = (-nside * g / 2,) * 3
    R = oc.analytic_randoms((nside,) * 3, origin, g, 1e6, p_ang, (0.0, 360.0), (-90.0, 90.0), p_z, z_range)
    assert abs(R.sum() / 1e6 - 1.0) < 0.01
    idx = np.indices(R.shape).reshape(3, -1).T
    centres = np.asarray(origin) + (idx + 0.5) * g
    rr = np.linalg.norm(centres, axis=1).reshape(R.shape)
    assert np.all(R[(rr < r0 - 1e-9) | (rr > r1 + 1e-9)] == 0.0)
