"""Equidistant (diagonal) n-point sums, Eq. ksinDiag, through the C ABI against
the FP64 oracle: streamed out of the inverse FFT (conker_convolve_diag, no maps
stored) and from stored maps (conker_contract_diag), n = 2 .. 5, on grids with
radix-2 and radix-3 axes up to 1024 cells long.

Error measure: max |got - ref| / max |ref| per (field, order).  Bars: float64
<= 1e-12; float32 <= 1e-5 (the map error of the FP32 transforms, ~1e-6 of the
largest map value, enters C^(n-1) at most n-1 times).
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TDT = {"f32": torch.float32, "f64": torch.float64}
TOL = {"f32": 1e-5, "f64": 1e-12}
DIMS = [(32, 32, 32), (64, 32, 96), (96, 64, 192), (32, 32, 1024), (64, 64, 384), (32, 64, 512)]
RADII = [0.5, 1.0, 2.0, 3.5, 5.0, 8.0, 11.0, 15.0]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


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


def _fields(dims, dt, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=dims)
    B = rng.poisson(2.0, size=dims).astype(np.float64)
    if dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    return A, B


def _oracle_diag(F, radii, n_max):
    out = np.zeros((n_max - 1, len(radii)))
    for m, r in enumerate(radii):
        c = oc.convolve_shell(F, r)
        for n in range(2, n_max + 1):
            out[n - 2, m] = oc.diagonal(F, c, n)
    return out


def _radii(dims):
    return [r for r in RADII if 2 * oc.shell_reach(r) + 1 <= min(dims)]


@pytest.mark.parametrize("dims", DIMS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_convolve_diag_vs_oracle(ck, ctx, dims, dt):
    radii = _radii(dims)
    _say("convolve_diag", dims, dt, radii)
    A, B = _fields(dims, dt, 31)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    ta = torch.from_numpy(A).to(DEV, TDT[dt])
    tb = torch.from_numpy(B).to(DEV, TDT[dt])
    oa, ob = ctx.convolve_diag(grid, ta, tb, ks, 5)
    ra, rb = _oracle_diag(A, radii, 5), _oracle_diag(B, radii, 5)
    oa, ob = oa.cpu().numpy(), ob.cpu().numpy()
    for k in range(4):
        ea, eb = relerr(oa[k], ra[k]), relerr(ob[k], rb[k])
        _say("  n=%d  a %.2e  b %.2e" % (k + 2, ea, eb))
        assert ea <= TOL[dt] and eb <= TOL[dt], (k + 2, ea, eb)


@pytest.mark.parametrize("dims", [(64, 32, 96), (32, 64, 512)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_contract_diag_vs_oracle(ck, ctx, dims, dt):
    radii = _radii(dims)
    _say("contract_diag", dims, dt)
    A, _ = _fields(dims, dt, 32)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    ta = torch.from_numpy(A).to(DEV, TDT[dt])
    maps, _ = ctx.convolve_shells(grid, ta, None, ks)
    ref = _oracle_diag(A, radii, 5)
    for n_max in (2, 3, 5):
        got = ctx.contract_diag(grid, ta, maps, n_max).cpu().numpy()
        assert got.shape == (n_max - 1, len(radii))
        for k in range(n_max - 1):
            assert relerr(got[k], ref[k]) <= TOL[dt], (n_max, k)


def test_convolve_diag_batches_single_field_and_full_tuples(ck, ctx):
    """Radius batches of 3 give the same sums; field_b = NULL; the diagonal of
    the full n = 3 and n = 4 outputs of conker_contract_npt matches."""
    dims = (64, 64, 64)
    radii = [1.0, 2.0, 3.0, 4.5, 6.0, 9.0, 13.0]
    A, B = _fields(dims, "f64", 33)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float64)
    ta, tb = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    full_a, full_b = ctx.convolve_diag(grid, ta, tb, ks, 4)
    os.environ["CONKER_RADIUS_BATCH"] = "3"
    try:
        part_a, part_b = ctx.convolve_diag(grid, ta, tb, ks, 4)
        solo, none = ctx.convolve_diag(grid, ta, None, ks, 4)
    finally:
        del os.environ["CONKER_RADIUS_BATCH"]
    assert none is None
    assert relerr(part_a.cpu().numpy(), full_a.cpu().numpy()) <= 1e-14
    assert relerr(part_b.cpu().numpy(), full_b.cpu().numpy()) <= 1e-14
    assert relerr(solo.cpu().numpy(), full_a.cpu().numpy()) <= 1e-14
    maps, _ = ctx.convolve_shells(grid, ta, None, ks)
    ns = len(radii)
    for n in (3, 4):
        W = ctx.contract_npt(grid, ta, maps, n, "f64").cpu().numpy()
        idx = {t: i for i, t in enumerate(oc.radius_tuples(ns, n))}
        diag = np.array([W[idx[(m,) * (n - 1)]] for m in range(ns)])
        assert relerr(full_a.cpu().numpy()[n - 2], diag) <= 1e-12


@pytest.mark.parametrize("path", ["f64", "f32"])
def test_npcf_diag_cube128(ck, ctx, path):
    w = synth.workload("cube512_ns20k_grid128")
    data, rand = w.make()
    D, wd, _ = oc.histogram(data.pos, None, w.origin, w.cell, w.dims)
    R, wr, _ = oc.histogram(rand.pos, None, w.origin, w.cell, w.dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    rc = [r / w.cell for r in w.radii]
    rd, rr = _oracle_diag(N, rc, 5), _oracle_diag(R, rc, 5)
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, TDT[path])
    out = ck.npcf_diag(ctx, grid, torch.from_numpy(data.pos).to(DEV), torch.from_numpy(rand.pos).to(DEV), ks, 5,
                       dtype=TDT[path])
    Wd, Wr, xi = (out[k].cpu().numpy() for k in ("W_delta", "W_rand_raw", "xi"))
    assert abs(out["alpha"].item() - alpha) <= 1e-15 * alpha
    for k in range(4):
        n = k + 2
        ed, er = relerr(Wd[k], rd[k]), relerr(Wr[k], rr[k])
        ex = relerr(xi[k], rd[k] / (alpha ** n * rr[k]))
        _say("  cube128 diag n=%d  W_delta %.2e  W_R %.2e  xi %.2e" % (n, ed, er, ex))
        assert ed <= TOL[path] and er <= TOL[path] and ex <= 10 * TOL[path]


def test_diag_argument_errors(ck, ctx):
    dims = (32, 32, 32)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, [2.0], torch.float64)
    f = torch.zeros(dims, dtype=torch.float64, device=DEV)
    with pytest.raises(ck.ConkerError):
        ctx.convolve_diag(grid, f, None, ks, 6)
    with pytest.raises(ck.ConkerError):
        ctx.convolve_diag(grid, f, None, ks, 1)
    maps = torch.zeros((1,) + dims, dtype=torch.float64, device=DEV)
    with pytest.raises(ck.ConkerError):
        ctx.contract_diag(grid, f, maps, 6)
    # a zero field gives zero sums
    oa, _ = ctx.convolve_diag(grid, f, None, ks, 5)
    assert np.all(oa.cpu().numpy() == 0.0)


@pytest.mark.parametrize("dims", [(96, 64, 96), (64, 32, 512)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_convolve_diag_sparse_support(ck, ctx, dims, dt):
    """Fields vanishing on many z-lines and whole x-slabs: only carrying lines
    are transformed back, the sums are unchanged."""
    rng = np.random.default_rng(42)
    nx, ny, nz = dims
    A, B = _fields(dims, dt, 43)
    x = np.arange(nx)[:, None]
    y = np.arange(ny)[None, :]
    keep = ((x - nx / 2) / (nx / 2)) ** 2 + ((y - ny / 2) / (ny / 2)) ** 2 <= 0.6
    keep[: nx // 5] = False
    keep &= rng.random(keep.shape) < 0.8
    A = A * keep[:, :, None]
    B = B * keep[:, :, None]
    radii = _radii(dims)
    _say("convolve_diag sparse", dims, dt, "carrying lines %.3f" % keep.mean())
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    oa, ob = ctx.convolve_diag(grid, torch.from_numpy(A).to(DEV, TDT[dt]), torch.from_numpy(B).to(DEV, TDT[dt]),
                               ks, 5)
    ra, rb = _oracle_diag(A, radii, 5), _oracle_diag(B, radii, 5)
    for k in range(4):
        ea, eb = relerr(oa.cpu().numpy()[k], ra[k]), relerr(ob.cpu().numpy()[k], rb[k])
        _say("  n=%d  a %.2e  b %.2e" % (k + 2, ea, eb))
        assert ea <= TOL[dt] and eb <= TOL[dt], (k + 2, ea, eb)
