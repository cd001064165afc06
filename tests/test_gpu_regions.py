"""Regions combined (Eq. ksi3combined), per-cell W_0 W_1 / <B_0 B_1> maps and
value histograms (Sec. 4.2) through the C ABI against the FP64 oracle.
Bars: float64 <= 1e-12 (elementwise relative to the largest value); the
histograms are integer counts and must match exactly.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


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


@pytest.mark.parametrize("n_regions", [1, 2, 5])
def test_ratio_combined(ck, ctx, n_regions):
    rng = np.random.default_rng(70 + n_regions)
    n, cnt = 3, 465
    Wd = rng.normal(size=(n_regions, cnt))
    Wr = rng.uniform(1.0, 2.0, size=(n_regions, cnt))
    al = rng.uniform(0.01, 0.05, size=n_regions)
    xi, num, den = ctx.ratio_combined(torch.from_numpy(Wd).to(DEV), torch.from_numpy(Wr).to(DEV),
                                      torch.from_numpy(al).to(DEV), n)
    rxi, rnum, rden = oc.combine_regions(list(Wd), list(Wr), list(al), n)
    assert relerr(num.cpu().numpy(), rnum) <= 1e-14
    assert relerr(den.cpu().numpy(), rden) <= 1e-14
    assert np.allclose(xi.cpu().numpy(), rxi, rtol=1e-13, atol=0)


def test_combined_caps_through_the_batch(ck, ctx):
    """Two caps of one survey run as two jobs; their combination equals the
    estimator of the union (same alpha by construction), within 1e-12."""
    dims, cell = (64, 64, 64), 1.0
    rng = np.random.default_rng(80)
    d1 = rng.uniform(2, 20, size=(3000, 3)).astype(np.float32)
    r1 = rng.uniform(2, 20, size=(30000, 3)).astype(np.float32)
    d2 = (rng.uniform(2, 20, size=(3000, 3)) + [36, 0, 0]).astype(np.float32)
    r2 = (rng.uniform(2, 20, size=(30000, 3)) + [36, 0, 0]).astype(np.float32)
    radii = [1.0, 2.0, 4.0, 6.0]
    grid = ck.Grid(dims, (0, 0, 0), cell)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float64)
    outs = [ck.npcf(ctx, grid, torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV), ks, 3)
            for d, r in ((d1, r1), (d2, r2))]
    Wd = torch.stack([o["W_delta"] for o in outs])
    Wr = torch.stack([o["W_rand_raw"] for o in outs])
    al = torch.cat([o["alpha"] for o in outs])
    xi, _, _ = ctx.ratio_combined(Wd, Wr, al, 3)
    ref = oc.npcf(np.concatenate([d1, d2]), np.concatenate([r1, r2]), dims, (0, 0, 0), cell, radii, 3)
    assert relerr(xi.cpu().numpy(), ref["xi"]) <= 1e-12


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_map_ratio_and_histogram(ck, ctx, dt):
    w = synth.workload("cube512_ns20k_grid128")
    data, rand = w.make()
    ref = oc.npcf(data.pos, rand.pos, w.dims, w.origin, w.cell, w.radii[:3], 2)
    tdt = torch.float64 if dt == "f64" else torch.float32
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ks, _ = ctx.make_shell_kernels(grid, w.radii[:3], tdt)
    out = ck.npcf(ctx, grid, torch.from_numpy(data.pos).to(DEV), torch.from_numpy(rand.pos).to(DEV), ks, 2,
                  precision="f64" if dt == "f64" else "f32", dtype=tdt, fused=False)
    maps = out["bufs"]["maps_N"]
    for m in range(3):
        got = ctx.map_ratio(grid, out["bufs"]["N"], maps[m], out["W_rand_raw"][m:m + 1], out["alpha"])
        exp = oc.map_ratio(ref["N"], ref["maps_N"][m], ref["W_rand_raw"][m], ref["alpha"])
        e = relerr(got.cpu().numpy(), exp)
        assert e <= (1e-12 if dt == "f64" else 1e-5), (m, e)
        # the average of the map is the 2pcf of that radius
        assert abs(float(got.double().mean()) - ref["xi"][m]) <= (1e-10 if dt == "f64" else 1e-4) * abs(ref["xi"][m])
    # histogram of oracle-made values (the same array on both sides), bit-exact counts
    vals = oc.map_ratio(ref["N"], ref["maps_N"][1], ref["W_rand_raw"][1], ref["alpha"]).ravel()
    vals = vals.astype(np.float32).astype(np.float64) if dt == "f32" else vals
    vals[::1000] = np.nan
    lo, hi = -5.0, 40.0
    counts = ctx.value_histogram(torch.from_numpy(vals).to(DEV, tdt), lo, hi, 90).cpu().numpy()
    assert counts.tolist() == oc.value_histogram(vals, lo, hi, 90).tolist()
    assert counts.sum() == vals.size


def test_histogram_errors_and_empty(ck, ctx):
    v = torch.zeros(0, dtype=torch.float32, device=DEV)
    assert ctx.value_histogram(v, 0.0, 1.0, 4).cpu().tolist() == [0] * 6
    with pytest.raises(ck.ConkerError):
        ctx.value_histogram(v, 1.0, 1.0, 4)
    with pytest.raises(ck.ConkerError):
        ctx.value_histogram(v, 0.0, 1.0, 0)
