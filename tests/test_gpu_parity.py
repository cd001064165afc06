"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Error measure for W (and maps): max |got - ref| / max |ref| over the outputs of
one call.  Bars: integer work (histograms of unit weights, shell sizes)
bit-exact; float64 path <= 1e-12; float32 / split-bf16 paths <= 1e-5.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


DEV = "cuda:0"
TDT = {"f32": torch.float32, "f64": torch.float64}


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def elementwise_relerr(got, ref):
    """max_t |got_t - ref_t| / |ref_t|, for sums that are positive tuple by tuple."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert np.all(ref > 0)
    return float((np.abs(got - ref) / ref).max())


def _gpu(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t if dtype is None else t.to(dtype)


# ---------------------------------------------------------------------------
# mapping
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_scatter_unit_weights_bit_exact(ck, ctx, dt):
    w = synth.workload("cube512_ns20k_grid128")
    data, rand = w.make()
    grid = ck.Grid(w.dims, w.origin, w.cell)
    for cat in (data, rand):
        _say("scatter unit", dt, len(cat))
        out = torch.zeros(w.dims, dtype=TDT[dt], device=DEV)
        wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
        nout = torch.zeros(1, dtype=torch.int64, device=DEV)
        ctx.grid_assign(grid, _gpu(cat.pos), None, out, wsum, nout)
        ref, rs, ro = oc.histogram(cat.pos, None, w.origin, w.cell, w.dims)
        assert np.array_equal(out.cpu().numpy().astype(np.float64), ref)
        assert wsum.item() == rs and nout.item() == ro


@pytest.mark.parametrize("dt,tol", [("f32", 2e-6), ("f64", 1e-13)])
def test_scatter_weighted_survey_cap(ck, ctx, dt, tol):
    w = synth.workload("cap512_ns800k_r30")
    data, rand = w.make(scale=0.02)
    grid = ck.Grid(w.dims, w.origin, w.cell)
    for cat in (data, rand):
        _say("scatter weighted", dt, len(cat))
        out = torch.zeros(w.dims, dtype=TDT[dt], device=DEV)
        wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
        nout = torch.zeros(1, dtype=torch.int64, device=DEV)
        ctx.grid_assign(grid, _gpu(cat.pos), _gpu(cat.w), out, wsum, nout)
        ref, rs, ro = oc.histogram(cat.pos, cat.w, w.origin, w.cell, w.dims)
        got = out.cpu().numpy().astype(np.float64)
        assert np.abs(got - ref).max() <= tol * ref.max()
        assert math.isclose(wsum.item(), rs, rel_tol=1e-12)
        assert nout.item() == ro == 0


@pytest.mark.parametrize("dims", [(128, 128, 128), (72, 64, 64)])
@pytest.mark.parametrize("dt,weighted,tol", [("f32", False, 0.0), ("f64", False, 0.0), ("f32", True, 2e-6),
                                             ("f64", True, 1e-13)])
def test_scatter_large_catalog(ck, ctx, dims, dt, weighted, tol):
    """Five million clustered points: 128^3 takes the brick-binned mapping,
    72 x 64 x 64 (not a whole number of bricks) the direct one.  The grid is
    accumulated into (pre-filled with 0.5); unit weights must count exactly."""
    n = 5_000_000
    pos = synth.neyman_scott_box(n, 300, 2.0, -3.0, 130.0, seed=171)
    pos[::100_003] = np.nan
    w = synth.lognormal_weights(n, 0.2, seed=172) if weighted else None
    grid = ck.Grid(dims, (0.0, 0.0, 0.0), 1.0)
    _say("scatter large", dims, dt, weighted)
    out = torch.full(dims, 0.5, dtype=TDT[dt], device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    nout = torch.zeros(1, dtype=torch.int64, device=DEV)
    ctx.grid_assign(grid, _gpu(pos), _gpu(w) if weighted else None, out, wsum, nout)
    ref, rs, ro = oc.histogram(pos, w, (0.0, 0.0, 0.0), 1.0, dims)
    got = out.cpu().numpy().astype(np.float64) - 0.5
    assert ro > 0 and nout.item() == ro
    if weighted:
        assert np.abs(got - ref).max() <= tol * ref.max()
        assert math.isclose(wsum.item(), rs, rel_tol=1e-12)
    else:
        assert np.array_equal(got, ref)
        assert wsum.item() == rs


@pytest.mark.parametrize("wscale", [1e-8, 1e-9])
@pytest.mark.parametrize("dt,tol", [("f32", 2e-6), ("f64", 1e-13)])
def test_scatter_binned_tiny_weights(ck, ctx, wscale, dt, tol):
    """Weights normalised to tiny values (as when a random catalog is scaled to
    sum to one) through the brick-binned mapping: per cell within the bar of
    max |ref|, and the grid total equal to the weight sum (a rounding bias in
    the brick sums would shift every cell the same way)."""
    n = 4_500_000
    dims = (128, 128, 128)
    pos = synth.neyman_scott_box(n, 300, 2.0, 0.0, 128.0, seed=181)
    w = (synth.lognormal_weights(n, 0.2, seed=182) * np.float32(wscale)).astype(np.float32)
    grid = ck.Grid(dims, (0.0, 0.0, 0.0), 1.0)
    _say("scatter binned tiny weights", wscale, dt)
    out = torch.zeros(dims, dtype=TDT[dt], device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.grid_assign(grid, _gpu(pos), _gpu(w), out, wsum)
    ref, rs, ro = oc.histogram(pos, w, (0.0, 0.0, 0.0), 1.0, dims)
    got = out.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref).max() / ref.max()
    bias = abs(got.sum() - rs) / rs
    _say("  max err %.3e of max, total %.3e" % (err, bias))
    assert ro == 0 and math.isclose(wsum.item(), rs, rel_tol=1e-12)
    assert err <= tol and bias <= tol


def test_scatter_rejects_outside_and_nonfinite(ck, ctx):
    dims, origin, cell = (32, 32, 32), (0.0, 0.0, 0.0), 1.0
    grid = ck.Grid(dims, origin, cell)
    pos = np.array([[1.5, 2.5, 3.5], [32.0, 1.0, 1.0], [-0.001, 1, 1], [5, 5, np.nan],
                    [31.999, 31.999, 31.999], [7, 7, 7]], dtype=np.float32)
    wts = np.array([1.0, 1.0, 1.0, 1.0, 2.0, np.inf], dtype=np.float32)
    out = torch.zeros(dims, dtype=torch.float64, device=DEV)
    wsum = torch.zeros(1, dtype=torch.float64, device=DEV)
    nout = torch.zeros(1, dtype=torch.int64, device=DEV)
    ctx.grid_assign(grid, _gpu(pos), _gpu(wts), out, wsum, nout)
    g = out.cpu().numpy()
    assert g[1, 2, 3] == 1.0 and g[31, 31, 31] == 2.0 and g.sum() == 3.0
    assert nout.item() == 4 and wsum.item() == 3.0


def test_scatter_empty_catalog_is_noop(ck, ctx):
    grid = ck.Grid((32, 32, 32), (0, 0, 0), 1.0)
    out = torch.zeros((32, 32, 32), dtype=torch.float32, device=DEV)
    ctx.grid_assign(grid, torch.zeros((0, 3), dtype=torch.float32, device=DEV), None, out)
    assert out.abs().sum().item() == 0.0


@pytest.mark.parametrize("dt,tol", [("f32", 1e-6), ("f64", 1e-15)])
def test_form_delta(ck, ctx, dt, tol):
    rng = np.random.default_rng(3)
    D = rng.integers(0, 5, size=(32, 32, 64)).astype(np.float64)
    R = rng.integers(0, 40, size=(32, 32, 64)).astype(np.float64)
    grid = ck.Grid((32, 32, 64), (0, 0, 0), 1.0)
    Dt, Rt = _gpu(D, TDT[dt]), _gpu(R, TDT[dt])
    ws = torch.tensor([D.sum(), R.sum()], dtype=torch.float64, device=DEV)
    alpha = torch.zeros(1, dtype=torch.float64, device=DEV)
    ctx.form_delta(grid, Dt, Rt, ws[0:1], ws[1:2], alpha)
    N, a = oc.density_deviation(D, R, D.sum(), R.sum())
    assert alpha.item() == a
    assert relerr(Dt.cpu().numpy(), N) <= tol


# ---------------------------------------------------------------------------
# kernels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(32, 32, 32), (64, 32, 128), (128, 128, 128), (96, 192, 96)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_shell_kernel_spectra(ck, ctx, dims, dt):
    cell = 2.0
    radii = [1.0, 2.0, 3.0, 5.0, 7.5, 9.0, 22.0]   # r = 0.5 .. 11 cells, odd count
    radii = [r for r in radii if 2 * oc.shell_reach(r / cell) + 1 <= min(dims)]
    _say("shells", dims, dt, radii)
    grid = ck.Grid(dims, (0, 0, 0), cell)
    ks, sizes = ctx.make_shell_kernels(grid, radii, TDT[dt])
    # stored octant layout: [radius][ky][kz][kx] (x fastest)
    ks = ks.cpu().numpy().reshape(len(radii), dims[1] // 2 + 1, dims[2] // 2 + 1, dims[0] // 2 + 1)
    ks = ks.transpose(0, 3, 1, 2)
    nc = np.prod(dims)
    for m, s in enumerate(radii):
        r = s / cell
        assert sizes[m] == len(oc.shell_offsets(r))
        ref = oc.shell_spectrum(r, dims).real[: dims[0] // 2 + 1, : dims[1] // 2 + 1, : dims[2] // 2 + 1] / nc
        tol = 1e-13 if dt == "f64" else 1e-7
        assert np.abs(ks[m] - ref).max() <= tol * sizes[m] / nc, (m, r)
        assert abs(ks[m][0, 0, 0] * nc - sizes[m]) <= (1e-9 if dt == "f64" else 1e-3)


def test_shell_radius_errors(ck, ctx):
    grid = ck.Grid((32, 32, 32), (0, 0, 0), 1.0)
    with pytest.raises(ck.ConkerError) as e:
        ctx.make_shell_kernels(grid, [16.0], torch.float64)
    assert "ERANGE" in str(e.value)
    with pytest.raises(ck.ConkerError) as e:
        ctx.make_shell_kernels(grid, [0.4], torch.float64)
    assert "ERANGE" in str(e.value)
    with pytest.raises(ck.ConkerError) as e:
        ctx.make_shell_kernels(ck.Grid((80, 80, 80), (0, 0, 0), 1.0), [3.0], torch.float64)
    assert "UNSUPPORTED" in str(e.value)


# ---------------------------------------------------------------------------
# convolution
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(32, 32, 32), (32, 64, 128), (128, 64, 32), (64, 64, 64), (96, 96, 96),
                                  (192, 96, 96), (96, 192, 384), (1024, 32, 32), (32, 1024, 64)])
@pytest.mark.parametrize("dt,tol", [("f64", 1e-12), ("f32", 3e-6)])
def test_convolve_shells_vs_oracle(ck, ctx, dims, dt, tol):
    rng = np.random.default_rng(11)
    A = rng.normal(size=dims)
    B = rng.poisson(3.0, size=dims).astype(np.float64)
    cell = 1.0
    radii = [1.0, 2.0, 3.0, 4.0, 6.0, 9.0, 13.0]
    radii = [r for r in radii if 2 * oc.shell_reach(r) + 1 <= min(dims)]
    _say("convolve", dims, dt, radii)
    grid = ck.Grid(dims, (0, 0, 0), cell)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    ma, mb = ctx.convolve_shells(grid, _gpu(A, TDT[dt]), _gpu(B, TDT[dt]), ks)
    ma, mb = ma.cpu().numpy(), mb.cpu().numpy()
    Af = A.astype(np.float32).astype(np.float64) if dt == "f32" else A
    Bf = B
    for m, r in enumerate(radii):
        ra, rb = oc.convolve_shell(Af, r), oc.convolve_shell(Bf, r)
        ea, eb = relerr(ma[m], ra), relerr(mb[m], rb)
        assert ea <= tol and eb <= tol, (m, r, ea, eb)


def test_convolve_single_field_and_one_radius(ck, ctx):
    dims = (64, 64, 64)
    rng = np.random.default_rng(12)
    A = rng.normal(size=dims)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, [5.0], torch.float64)
    ma, mb = ctx.convolve_shells(grid, _gpu(A), None, ks)
    assert mb is None
    assert relerr(ma.cpu().numpy()[0], oc.convolve_shell(A, 5.0)) <= 1e-12


@pytest.mark.parametrize("ns,dims", [(2, (64, 96, 32)), (5, (64, 96, 32)), (8, (64, 96, 32)), (5, (1024, 32, 32))])
@pytest.mark.parametrize("dt,tol", [("f64", 1e-12), ("f32", 3e-6)])
def test_convolve_single_field_radius_pairs(ck, ctx, ns, dims, dt, tol):
    """One field: radii travel in pairs (C_a + i C_b through one inverse
    transform); odd counts leave a lone last radius; batches of one pair give
    bitwise the same maps."""
    import os
    radii = [1.0, 2.0, 3.5, 5.0, 7.0, 9.0, 12.0, 15.0][:ns]
    rng = np.random.default_rng(14)
    A = rng.normal(size=dims)
    Af = A.astype(np.float32).astype(np.float64) if dt == "f32" else A
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    maps, none = ctx.convolve_shells(grid, _gpu(A, TDT[dt]), None, ks)
    assert none is None
    got = maps.cpu().numpy()
    for m, r in enumerate(radii):
        e = relerr(got[m], oc.convolve_shell(Af, r))
        assert e <= tol, (m, r, e)
    os.environ["CONKER_RADIUS_BATCH"] = "1"
    try:
        maps1, _ = ctx.convolve_shells(grid, _gpu(A, TDT[dt]), None, ks)
    finally:
        del os.environ["CONKER_RADIUS_BATCH"]
    assert np.array_equal(maps1.cpu().numpy(), got)


def test_convolve_integer_field_equals_direct_shell_sums(ck, ctx):
    dims = (64, 64, 64)
    rng = np.random.default_rng(13)
    A = rng.integers(-2, 3, size=dims).astype(np.float64)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, [7.0, 20.0], torch.float64)
    ma, _ = ctx.convolve_shells(grid, _gpu(A), None, ks)
    ma = ma.cpu().numpy()
    cells = rng.integers(0, 64, size=(200, 3))
    for m, r in enumerate([7.0, 20.0]):
        direct = oc.direct_shell_sum(A, r, cells)
        got = ma[m][cells[:, 0], cells[:, 1], cells[:, 2]]
        assert np.abs(got - direct).max() < 1e-9


# ---------------------------------------------------------------------------
# summation
# ---------------------------------------------------------------------------

CONTRACT_CASES = [
    # (prec, n, n_radii, dims)
    ("f64", 2, 7, (32, 32, 32)),
    ("f64", 3, 7, (32, 32, 32)),
    ("f64", 3, 33, (32, 32, 64)),
    ("f64", 4, 9, (32, 32, 32)),
    ("f64", 5, 6, (32, 32, 32)),
    ("f32", 2, 30, (32, 32, 32)),
    ("f32", 3, 30, (32, 64, 64)),
    ("f32", 3, 40, (32, 32, 32)),
    ("f32", 4, 9, (32, 32, 32)),
    ("f32", 5, 6, (32, 32, 32)),
    ("split_bf16", 2, 30, (32, 32, 32)),
    ("split_bf16", 3, 30, (32, 64, 64)),
    ("split_bf16", 3, 40, (32, 32, 32)),
    ("split_bf16", 4, 9, (32, 32, 32)),
    ("split_bf16", 5, 6, (32, 32, 32)),
    # operand-sharing kernel with several tiles and tile groups
    ("split_bf16", 4, 30, (32, 32, 32)),
    ("f32", 4, 30, (32, 32, 32)),
    ("split_bf16", 5, 20, (32, 32, 32)),
    ("f32", 5, 20, (32, 32, 32)),
    ("split_bf16", 5, 30, (32, 32, 32)),
    ("split_bf16", 3, 64, (32, 32, 32)),
    ("f64", 4, 30, (32, 32, 32)),
    ("f64", 5, 20, (32, 32, 32)),
    # split float16 with power-of-two operand scaling
    ("split_f16", 2, 30, (32, 32, 32)),
    ("split_f16", 3, 30, (32, 64, 64)),
    ("split_f16", 3, 40, (32, 32, 32)),
    ("split_f16", 4, 9, (32, 32, 32)),
    ("split_f16", 4, 30, (32, 32, 32)),
    ("split_f16", 5, 6, (32, 32, 32)),
    ("split_f16", 5, 20, (32, 32, 32)),
]


@pytest.mark.parametrize("prec,n,ns,dims", CONTRACT_CASES)
def test_contract_vs_oracle(ck, ctx, prec, n, ns, dims):
    _say("contract", prec, n, ns, dims)
    rng = np.random.default_rng(100 + n * 7 + ns)
    F = rng.normal(size=dims)
    maps = rng.normal(size=(ns,) + dims) + 0.3
    dt = torch.float64 if prec == "f64" else torch.float32
    if dt == torch.float32:
        F = F.astype(np.float32).astype(np.float64)
        maps = maps.astype(np.float32).astype(np.float64)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    W = ctx.contract_npt(grid, _gpu(F, dt), _gpu(maps, dt), n, prec).cpu().numpy()
    ref = oc.contract(F, maps, n)
    err = relerr(W, ref)
    bad = np.argsort(-np.abs(W - ref))[:5]
    _say("  err %.3e worst tuples %s" % (err, [oc.radius_tuples(ns, n)[i] for i in bad]))
    assert err <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_split_f16_wide_dynamic_range(ck, ctx, n):
    """Maps and fields spanning many binades (count-like maps of very different
    sizes per radius, a field with values from 1e-6 to 1e4): the per-map
    power-of-two scaling keeps every operand inside the float16 range."""
    dims = (32, 32, 32)
    ns = 12
    rng = np.random.default_rng(200 + n)
    F = rng.normal(size=dims) * np.exp(rng.uniform(np.log(1e-6), np.log(1e4), size=dims))
    scale = np.exp(np.linspace(np.log(1e-3), np.log(3e4), ns))[:, None, None, None]
    maps = (rng.poisson(5.0, size=(ns,) + dims) + 0.5) * scale
    F = F.astype(np.float32).astype(np.float64)
    maps = maps.astype(np.float32).astype(np.float64)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    W = ctx.contract_npt(grid, _gpu(F, torch.float32), _gpu(maps, torch.float32), n, "split_f16").cpu().numpy()
    ref = oc.contract(F, maps, n)
    # per tuple, relative to the largest |term| sum of that tuple's scale
    mag = oc.contract(np.abs(F), maps, n)
    err = float(np.max(np.abs(W - ref) / mag))
    _say("split_f16 wide range n=%d: max |err| / sum|terms| %.3e" % (n, err))
    assert err <= 1e-5


def _block_sparse_field(dims, rng, dt):
    """F zero (either sign) on about 70 % of the 64-cell blocks of the flat
    grid, with a single non-zero cell in some of those, and a ragged last block
    when the cell count is not a multiple of 64."""
    F = rng.normal(size=dims)
    flat = F.reshape(-1)
    nblk = -(-flat.size // 64)
    for b in np.flatnonzero(rng.random(nblk) < 0.7):
        seg = flat[64 * b:64 * b + 64]
        seg[:] = -0.0 if b % 3 == 0 else 0.0
        if b % 5 == 0:
            seg[rng.integers(len(seg))] = rng.normal()
    if dt == torch.float32:
        F = F.astype(np.float32).astype(np.float64)
    return F


SPARSE_CONTRACT_CASES = [
    # 2.5 workgroups of the block marking (2048 blocks each)
    ("f64", 2, 8, (64, 64, 80)),
    ("split_bf16", 2, 8, (64, 64, 80)),
    ("f64", 3, 12, (64, 64, 80)),
    ("f32", 3, 30, (64, 64, 80)),
    ("split_bf16", 3, 30, (64, 64, 80)),
    ("split_f16", 3, 30, (64, 64, 80)),
    ("split_bf16", 4, 9, (64, 64, 80)),
    ("split_f16", 4, 12, (64, 64, 80)),
    ("f32", 5, 6, (64, 64, 80)),
    ("f64", 4, 6, (64, 64, 80)),
    # 720 cells: the last 64-cell block holds 16
    ("f64", 2, 8, (3, 5, 48)),
    ("f64", 3, 8, (3, 5, 48)),
    ("f32", 3, 8, (3, 5, 48)),
    ("split_bf16", 3, 8, (3, 5, 48)),
    ("split_f16", 3, 8, (3, 5, 48)),
]


@pytest.mark.parametrize("prec,n,ns,dims", SPARSE_CONTRACT_CASES)
def test_contract_block_sparse_field_vs_oracle(ck, ctx, prec, n, ns, dims):
    """Only the 64-cell blocks where F is non-zero are summed: the result is the
    full sum over every cell."""
    _say("contract block-sparse", prec, n, ns, dims)
    rng = np.random.default_rng(300 + n * 11 + ns)
    dt = torch.float64 if prec == "f64" else torch.float32
    F = _block_sparse_field(dims, rng, dt)
    maps = rng.normal(size=(ns,) + dims) + 0.3
    if dt == torch.float32:
        maps = maps.astype(np.float32).astype(np.float64)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    W = ctx.contract_npt(grid, _gpu(F, dt), _gpu(maps, dt), n, prec).cpu().numpy()
    ref = oc.contract(F, maps, n)
    err = relerr(W, ref)
    _say("  err %.3e" % err)
    assert err <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec,n", [("f64", 2), ("f64", 3), ("split_bf16", 3), ("split_f16", 4)])
def test_contract_zero_field_gives_zero(ck, ctx, prec, n):
    """A field that is zero everywhere (no block to sum) gives exactly zero."""
    dims = (32, 32, 32)
    dt = torch.float64 if prec == "f64" else torch.float32
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    F = torch.zeros(dims, dtype=dt, device=DEV)
    M = torch.ones((6,) + dims, dtype=dt, device=DEV)
    W = ctx.contract_npt(grid, F, M, n, prec).cpu().numpy()
    assert W.shape == (oc.num_tuples(6, n),) and np.all(W == 0.0)


def test_contract_argument_errors(ck, ctx):
    grid = ck.Grid((32, 32, 32), (0, 0, 0), 1.0)
    F = torch.zeros((32, 32, 32), dtype=torch.float32, device=DEV)
    M = torch.zeros((3, 32, 32, 32), dtype=torch.float32, device=DEV)
    with pytest.raises(ck.ConkerError):
        ctx.contract_npt(grid, F, M, 3, "f64")          # float64 summation on float32 maps
    with pytest.raises(ck.ConkerError):
        ctx.contract_npt(grid, F, M, 6, "f32")          # order outside 2..5


# ---------------------------------------------------------------------------
# end to end
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cube128_ref():
    w = synth.workload("cube512_ns20k_grid128")
    data, rand = w.make()
    refs = {n: oc.npcf(data.pos, rand.pos, w.dims, w.origin, w.cell, w.radii, n) for n in (2, 3)}
    return w, data, rand, refs


@pytest.mark.parametrize("n", [3, 4])
@pytest.mark.parametrize("path,prec,tol", [("f64", "f64", 1e-12), ("f32", "split_f16", 1e-5)])
def test_end_to_end_cube128_field_at_a_time(ck, ctx, cube128_ref, n, path, prec, tol):
    w, data, rand, refs = cube128_ref
    ref = refs[n] if n in refs else oc.npcf(data.pos, rand.pos, w.dims, w.origin, w.cell, w.radii, n)
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, TDT[path])
    out = ck.npcf(ctx, grid, _gpu(data.pos), _gpu(rand.pos), ks, n, precision=prec, dtype=TDT[path],
                  fused=False, field_at_a_time=True)
    assert "maps_R" not in out["bufs"]
    ed = relerr(out["W_delta"].cpu().numpy(), ref["W_delta"])
    er = relerr(out["W_rand_raw"].cpu().numpy(), ref["W_rand_raw"])
    _say("  field at a time n=%d %s: W_delta %.3e  W_R %.3e" % (n, prec, ed, er))
    assert ed <= tol and er <= tol


@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("path,prec,tol", [("f64", "f64", 1e-12), ("f32", "f32", 1e-5),
                                           ("f32", "split_bf16", 1e-5)])
def test_end_to_end_cube128(ck, ctx, cube128_ref, n, path, prec, tol):
    w, data, rand, refs = cube128_ref
    ref = refs[n]
    _say("end-to-end cube128", n, path, prec)
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, TDT[path])
    out = ck.npcf(ctx, grid, _gpu(data.pos), _gpu(rand.pos), ks, n, precision=prec, dtype=TDT[path])
    ed = relerr(out["W_delta"].cpu().numpy(), ref["W_delta"])
    er = relerr(out["W_rand_raw"].cpu().numpy(), ref["W_rand_raw"])
    ex = relerr(out["xi"].cpu().numpy(), ref["xi"])
    _say("  W_delta %.3e  W_R %.3e  xi %.3e" % (ed, er, ex))
    assert abs(out["alpha"].item() - ref["alpha"]) <= 1e-15 * ref["alpha"]
    assert ed <= tol and er <= tol and ex <= 10 * tol


# ---------------------------------------------------------------------------
# fused convolution + summation (maps never stored)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def line512_fields():
    rng = np.random.default_rng(21)
    dims = (32, 64, 512)
    A = rng.normal(size=dims)
    B = rng.poisson(2.0, size=dims).astype(np.float64)
    radii = [0.5 * k for k in range(1, 31)]      # 0.5 .. 15 cells: half-integer radii included
    A32 = A.astype(np.float32).astype(np.float64)
    B32 = B.astype(np.float32).astype(np.float64)
    maps_a = oc.convolve_shells(A32, radii)
    maps_b = oc.convolve_shells(B32, radii)
    return dims, radii, A32, B32, maps_a, maps_b


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
@pytest.mark.parametrize("n", [2, 3])
@pytest.mark.parametrize("ns", [30, 7, 1])
def test_fused_convolve_contract_vs_oracle(ck, ctx, line512_fields, prec, n, ns):
    dims, radii, A, B, maps_a, maps_b = line512_fields
    _say("fused", prec, n, ns)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii[:ns], torch.float32)
    Wa, Wb = ctx.convolve_contract(grid, _gpu(A, torch.float32), _gpu(B, torch.float32), ks, n, prec)
    ra = oc.contract(A, maps_a[:ns], n)
    rb = oc.contract(B, maps_b[:ns], n)
    ea, eb = relerr(Wa.cpu().numpy(), ra), relerr(Wb.cpu().numpy(), rb)
    _say("  err a %.3e b %.3e" % (ea, eb))
    assert ea <= 1e-5 and eb <= 1e-5


def test_convolve_contract_single_field_and_routes(ck, ctx, line512_fields):
    """One field; the fused kernel (n = 3), the workspace maps (n = 4, and a z axis of
    256 cells), and argument errors."""
    dims, radii, A, B, maps_a, maps_b = line512_fields
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii[:5], torch.float32)
    Wa, Wb = ctx.convolve_contract(grid, _gpu(A, torch.float32), None, ks, 3, "split_bf16")
    assert Wb is None
    assert relerr(Wa.cpu().numpy(), oc.contract(A, maps_a[:5], 3)) <= 1e-5
    W4, _ = ctx.convolve_contract(grid, _gpu(A, torch.float32), None, ks, 4, "split_bf16")
    assert relerr(W4.cpu().numpy(), oc.contract(A, maps_a[:5], 4)) <= 1e-5
    rng = np.random.default_rng(23)
    A2 = rng.normal(size=(32, 32, 256)).astype(np.float32).astype(np.float64)
    g2 = ck.Grid((32, 32, 256), (0, 0, 0), 1.0)
    ks2, _ = ctx.make_shell_kernels(g2, radii[:3], torch.float32)
    W2, _ = ctx.convolve_contract(g2, _gpu(A2, torch.float32), None, ks2, 3, "split_bf16")
    assert relerr(W2.cpu().numpy(), oc.contract(A2, oc.convolve_shells(A2, radii[:3]), 3)) <= 1e-5
    with pytest.raises(ck.ConkerError):
        ctx.convolve_contract(grid, _gpu(A, torch.float32), None, ks, 6, "split_bf16")   # n outside 2..5
    with pytest.raises(ck.ConkerError):
        ctx.convolve_contract(grid, _gpu(A, torch.float32), None, ks, 3, "f64")          # f64 sums, f32 field


WORKSPACE_CASES = [
    ("f64", 2, 30), ("f64", 3, 30), ("f64", 4, 10), ("f64", 5, 6),
    ("f32", 4, 12), ("split_bf16", 4, 12), ("split_f16", 4, 12), ("split_f16", 3, 30), ("split_bf16", 5, 6),
]


@pytest.mark.parametrize("prec,n,ns", WORKSPACE_CASES)
def test_convolve_contract_workspace_maps_sparse_vs_oracle(ck, ctx, sparse512_fields, prec, n, ns):
    """Orders and precisions beyond the fused kernel: the maps of the carrying lines only, in
    the context's workspace, on fields zero outside a cylinder of lines and on whole slabs."""
    dims, radii, A, B, keep, maps_a, maps_b = sparse512_fields
    dt = torch.float64 if prec == "f64" else torch.float32
    _say("workspace maps", prec, n, ns)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii[:ns], dt)
    Wa, Wb = ctx.convolve_contract(grid, _gpu(A, dt), _gpu(B, dt), ks, n, prec)
    ref_a, ref_b = oc.contract(A, maps_a[:ns], n), oc.contract(B, maps_b[:ns], n)
    # A is zero-mean noise (its sums cancel), B one-signed: both against max |W|,
    # B also tuple by tuple
    ea = relerr(Wa.cpu().numpy(), ref_a)
    eb = relerr(Wb.cpu().numpy(), ref_b)
    eb_el = elementwise_relerr(Wb.cpu().numpy(), ref_b)
    _say("  err a %.3e b %.3e (b per tuple %.3e)" % (ea, eb, eb_el))
    tol = 1e-12 if prec == "f64" else 1e-5
    assert ea <= tol and eb <= tol and eb_el <= tol


def test_fused_matches_separate_calls_bitwise_order_free(ck, ctx, line512_fields):
    """The fused pass and convolve_shells + contract_npt agree to float32 rounding."""
    dims, radii, A, B, maps_a, maps_b = line512_fields
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
    At, Bt = _gpu(A, torch.float32), _gpu(B, torch.float32)
    Wa, Wb = ctx.convolve_contract(grid, At, Bt, ks, 3, "split_bf16")
    ma, mb = ctx.convolve_shells(grid, At, Bt, ks)
    Sa = ctx.contract_npt(grid, At, ma, 3, "split_bf16")
    Sb = ctx.contract_npt(grid, Bt, mb, 3, "split_bf16")
    assert relerr(Wa.cpu().numpy(), Sa.cpu().numpy()) <= 2e-6
    assert relerr(Wb.cpu().numpy(), Sb.cpu().numpy()) <= 2e-6


# ---------------------------------------------------------------------------
# fields that vanish on many z-lines (survey-shaped support): the fused pass
# transforms only lines that carry field; results must not change
# ---------------------------------------------------------------------------

def _sparse_support(dims, seed):
    """Fields zero outside an elliptic cylinder of lines and on whole x-slabs."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    A = rng.normal(size=dims)
    B = rng.poisson(2.0, size=dims).astype(np.float64)
    x = np.arange(nx)[:, None]
    y = np.arange(ny)[None, :]
    keep = ((x - nx / 2) / (nx / 2)) ** 2 + ((y - ny / 2) / (ny / 2)) ** 2 <= 0.7
    keep[: nx // 6] = False
    keep[nx - nx // 8:] = False
    A *= keep[:, :, None]
    B *= keep[:, :, None]
    B[:, :, : nz // 3] = 0.0       # lines of B vanish partly, never wholly where A is kept
    A = A.astype(np.float32).astype(np.float64)
    return A, B, keep


@pytest.fixture(scope="module")
def sparse512_fields():
    dims = (64, 64, 512)
    A, B, keep = _sparse_support(dims, 41)
    radii = [0.5 * k for k in range(1, 31)]
    return dims, radii, A, B, keep, oc.convolve_shells(A, radii), oc.convolve_shells(B, radii)


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
@pytest.mark.parametrize("n", [2, 3])
def test_fused_sparse_support_vs_oracle(ck, ctx, sparse512_fields, prec, n):
    dims, radii, A, B, keep, maps_a, maps_b = sparse512_fields
    _say("fused sparse support", prec, n, "carrying lines %.3f" % keep.mean())
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
    Wa, Wb = ctx.convolve_contract(grid, _gpu(A, torch.float32), _gpu(B, torch.float32), ks, n, prec)
    ref_a, ref_b = oc.contract(A, maps_a, n), oc.contract(B, maps_b, n)
    # A is zero-mean noise (its sums cancel), B one-signed: both against max |W|,
    # B also tuple by tuple
    ea = relerr(Wa.cpu().numpy(), ref_a)
    eb = relerr(Wb.cpu().numpy(), ref_b)
    eb_el = elementwise_relerr(Wb.cpu().numpy(), ref_b)
    _say("  err a %.3e b %.3e (b per tuple %.3e)" % (ea, eb, eb_el))
    assert ea <= 1e-5 and eb <= 1e-5 and eb_el <= 1e-5


@pytest.mark.parametrize("prec", ["split_bf16", "f32"])
def test_fused_sparse_support_nonnegative(ck, ctx, sparse512_fields, prec):
    """The same support with a field of one sign (no cancellation): 1e-5 of max |W|."""
    dims, radii, A, B, keep, maps_a, maps_b = sparse512_fields
    P = np.abs(A)
    maps_p = oc.convolve_shells(P, radii[:12])
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii[:12], torch.float32)
    Wp, _ = ctx.convolve_contract(grid, _gpu(P, torch.float32), None, ks, 3, prec)
    e = relerr(Wp.cpu().numpy(), oc.contract(P, maps_p, 3))
    _say("  nonnegative sparse, err %.3e" % e)
    assert e <= 1e-5


def test_fused_zero_fields_give_zero(ck, ctx, sparse512_fields):
    dims, radii, A, B, keep, maps_a, maps_b = sparse512_fields
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii[:6], torch.float32)
    z = torch.zeros(dims, dtype=torch.float32, device=DEV)
    Wa, Wb = ctx.convolve_contract(grid, z, z.clone(), ks, 3, "split_bf16")
    assert np.all(Wa.cpu().numpy() == 0.0) and np.all(Wb.cpu().numpy() == 0.0)
    # one field empty, the other sparse: the empty one still sums to exactly zero
    Wa, Wb = ctx.convolve_contract(grid, _gpu(A, torch.float32), z, ks, 3, "split_bf16")
    assert np.all(Wb.cpu().numpy() == 0.0)
    assert relerr(Wa.cpu().numpy(), oc.contract(A, maps_a[:6], 3)) <= 1e-5


@pytest.mark.parametrize("fn", ["npcf", "npcf_diag", "npcf_pair2"])
def test_outside_tracers_raise_unless_allowed(ck, ctx, fn):
    """Out-of-grid and non-finite tracers are counted by the mapping; the
    Python entry points raise unless they are explicitly allowed, and then the
    result equals that of the catalog without them."""
    dims = (32, 32, 32)
    rng = np.random.default_rng(140)
    d = rng.uniform(0, 32, size=(500, 3)).astype(np.float32)
    r = rng.uniform(0, 32, size=(5000, 3)).astype(np.float32)
    bad = np.array([[40.0, 1.0, 1.0], [np.nan, 2.0, 2.0], [3.0, -0.5, 3.0]], dtype=np.float32)
    d2 = np.concatenate([d, bad[:2]])
    r2 = np.concatenate([r, bad[2:]])
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, [2.0, 3.0, 5.0], torch.float64)
    call = {"npcf": lambda a, b, **kw: ck.npcf(ctx, grid, a, b, ks, 3, **kw),
            "npcf_diag": lambda a, b, **kw: ck.npcf_diag(ctx, grid, a, b, ks, 3, **kw),
            "npcf_pair2": lambda a, b, **kw: ck.npcf_pair2(ctx, grid, a, b, ks, **kw)}[fn]
    base = call(_gpu(d), _gpu(r))
    assert base["n_outside"].cpu().tolist() == [0, 0]
    with pytest.raises(ck.ConkerError) as e:
        call(_gpu(d2), _gpu(r2))
    assert "allow_outside" in str(e.value)
    out = call(_gpu(d2), _gpu(r2), allow_outside=True)
    assert out["n_outside"].cpu().tolist() == [2, 1]
    for k in ("W_delta", "W_rand_raw", "xi"):
        assert relerr(out[k].cpu().numpy(), base[k].cpu().numpy()) <= 1e-15, k
