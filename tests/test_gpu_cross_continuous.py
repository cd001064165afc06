"""Cross-correlation (Sec. 2.8), continuous delta fields (Sec. 2.7) and the
n = 2 Fourier-space form, through the C ABI against the FP64 oracle.

Error measure: max |got - ref| / max |ref| over one output vector.  Bars:
float64 <= 1e-12; float32 / split-bf16 <= 1e-5; delta fields elementwise
(float64 <= 1e-15 relative, float32 within one float32 rounding of the
float64 value).
"""
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


def _gpu(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, TDT[dt])


def _fields(dims, dt, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=dims) + 0.3
    B = rng.poisson(2.0, size=dims).astype(np.float64)
    if dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
    return A, B


# ---------------------------------------------------------------------------
# n = 2 from the spectra
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dims", [(32, 32, 32), (64, 96, 32), (96, 64, 192), (32, 32, 1024), (64, 32, 512)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_pair_spectral_vs_oracle(ck, ctx, dims, dt):
    radii = [r for r in (0.5, 1.0, 2.0, 3.5, 6.0, 9.0, 15.0) if 2 * oc.shell_reach(r) + 1 <= min(dims)]
    _say("pair_spectral", dims, dt, radii)
    A, B = _fields(dims, dt, 51)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    aa, bb, ab = ctx.pair_spectral(grid, _gpu(A, dt), _gpu(B, dt), ks)
    mA, mB = oc.convolve_shells(A, radii), oc.convolve_shells(B, radii)
    ea = relerr(aa.cpu().numpy(), oc.contract(A, mA, 2))
    eb = relerr(bb.cpu().numpy(), oc.contract(B, mB, 2))
    ex = relerr(ab.cpu().numpy(), oc.contract(A, mB, 2))
    _say("  aa %.2e  bb %.2e  ab %.2e" % (ea, eb, ex))
    assert ea <= TOL[dt] and eb <= TOL[dt] and ex <= TOL[dt]
    # single field
    aa1, none_b, none_ab = ctx.pair_spectral(grid, _gpu(A, dt), None, ks)
    assert none_b is None and none_ab is None
    assert relerr(aa1.cpu().numpy(), aa.cpu().numpy()) <= (1e-14 if dt == "f64" else 1e-6)


# ---------------------------------------------------------------------------
# continuous delta fields
# ---------------------------------------------------------------------------

def _continuous_fields(dims, seed):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.5, 2.0, size=dims)
    x = np.arange(dims[0])[:, None, None]
    R = R * (x < 3 * dims[0] // 4)            # no random coverage in the last quarter of x
    D = R * (1.0 + 0.3 * rng.normal(size=dims))
    return D, R


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_delta_field_elementwise(ck, ctx, dt):
    dims = (32, 64, 96)
    D, R = _continuous_fields(dims, 52)
    if dt == "f32":
        D = D.astype(np.float32).astype(np.float64)
        R = R.astype(np.float32).astype(np.float64)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    got = ctx.delta_field(grid, _gpu(D, dt), _gpu(R, dt)).cpu().numpy().astype(np.float64)
    ref = oc.delta_field(D, R)
    assert np.all(got[R == 0] == 0.0)
    if dt == "f64":
        assert np.all(np.abs(got - ref) <= 1e-15 * np.maximum(np.abs(ref), 1e-300) + 1e-300)
    else:
        assert np.array_equal(got, ref.astype(np.float32).astype(np.float64))
    alpha = torch.tensor([2.0], dtype=torch.float64, device=DEV)
    got2 = ctx.delta_field(grid, _gpu(D, dt), _gpu(R, dt), alpha).cpu().numpy().astype(np.float64)
    ref2 = oc.delta_field(D, 2.0 * R)
    assert relerr(got2, ref2) <= (1e-15 if dt == "f64" else 1e-7)


@pytest.mark.parametrize("dims,path", [((64, 32, 96), "f64"), ((64, 32, 512), "f64"), ((64, 32, 512), "mixed")])
@pytest.mark.parametrize("n", [2, 3])
def test_npcf_continuous_vs_oracle(ck, ctx, dims, path, n):
    D, R = _continuous_fields(dims, 53)
    dt = "f64" if path == "f64" else "f32"
    if dt == "f32":
        D = D.astype(np.float32).astype(np.float64)
        R = R.astype(np.float32).astype(np.float64)
    radii = [1.0, 2.0, 3.0, 5.0, 8.0, 12.0]
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    prec = "f64" if path == "f64" else "split_bf16"
    out = ck.npcf_continuous(ctx, grid, _gpu(D, dt), _gpu(R, dt), ks, n, precision=prec)
    delta = oc.delta_field(D, R)
    if dt == "f32":
        delta = delta.astype(np.float32).astype(np.float64)   # the GPU field is rounded once to float32
    ref = oc.contract(delta, oc.convolve_shells(delta, radii), n)
    e = relerr(out["xi"].cpu().numpy(), ref)
    _say("continuous", dims, path, n, "%.2e" % e)
    assert e <= TOL[dt]


# ---------------------------------------------------------------------------
# cross-correlation of two tracers
# ---------------------------------------------------------------------------

def _two_tracers(box, seed):
    d0 = synth.neyman_scott_box(6000, 120, 2.0, 0.0, box, seed)
    d1 = synth.neyman_scott_box(4000, 60, 3.0, 0.0, box, seed + 1)
    r = synth.uniform_box(60000, 0.0, box, seed + 2)
    w0 = synth.lognormal_weights(len(d0), 0.2, seed + 3)
    return d0, d1, r, w0


@pytest.mark.parametrize("dims,path,n", [((64, 64, 96), "f64", 2), ((64, 64, 96), "f64", 3),
                                         ((32, 64, 512), "f64", 3), ((32, 64, 512), "mixed", 2),
                                         ((32, 64, 512), "mixed", 3)])
def test_npcf_cross_vs_oracle(ck, ctx, dims, path, n):
    box = float(min(dims)) - 1.0
    d0, d1, r, w0 = _two_tracers(box, 60)
    radii = [1.0, 2.0, 3.0, 5.0, 7.0, 10.0]
    ref = oc.npcf_cross(d0, d1, r, dims, (0, 0, 0), 1.0, radii, n, data0_w=w0)
    dt = "f64" if path == "f64" else "f32"
    prec = "f64" if path == "f64" else "split_bf16"
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    out = ck.npcf_cross(ctx, grid, torch.from_numpy(d0).to(DEV), torch.from_numpy(d1).to(DEV),
                        torch.from_numpy(r).to(DEV), ks, n, data0_w=torch.from_numpy(w0).to(DEV),
                        precision=prec, dtype=TDT[dt])
    ec = relerr(out["W_cross"].cpu().numpy(), ref["W_cross"])
    er = relerr(out["W_rand_raw"].cpu().numpy(), ref["W_rand_raw"])
    ex = relerr(out["xi"].cpu().numpy(), ref["xi"])
    _say("cross", dims, path, n, "W %.2e  W_R %.2e  xi %.2e" % (ec, er, ex))
    a = out["alpha"].cpu().numpy()
    assert abs(a[0] - ref["alpha0"]) <= 1e-14 * ref["alpha0"] and abs(a[1] - ref["alpha1"]) <= 1e-14 * ref["alpha1"]
    assert ec <= TOL[dt] and er <= TOL[dt] and ex <= 10 * TOL[dt]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_convolve_diag_cross_vs_oracle(ck, ctx, dt):
    dims = (64, 32, 96)
    A, B = _fields(dims, dt, 54)
    C0 = np.abs(np.random.default_rng(55).normal(size=dims))
    if dt == "f32":
        C0 = C0.astype(np.float32).astype(np.float64)
    radii = [1.0, 2.0, 4.0, 7.0, 11.0]
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, radii, TDT[dt])
    oa, ob = ctx.convolve_diag(grid, _gpu(A, dt), _gpu(B, dt), ks, 4, centre_a=_gpu(C0, dt), centre_b=_gpu(A, dt))
    ra, rb = np.zeros((3, len(radii))), np.zeros((3, len(radii)))
    for m, r in enumerate(radii):
        cA, cB = oc.convolve_shell(A, r), oc.convolve_shell(B, r)
        for n in (2, 3, 4):
            ra[n - 2, m], rb[n - 2, m] = oc.diagonal(C0, cA, n), oc.diagonal(A, cB, n)
    oa, ob = oa.cpu().numpy(), ob.cpu().numpy()
    for k in range(3):
        ea, eb = relerr(oa[k], ra[k]), relerr(ob[k], rb[k])
        _say("  diag cross n=%d  a %.2e  b %.2e" % (k + 2, ea, eb))
        assert ea <= TOL[dt] and eb <= TOL[dt]


def test_cross_argument_errors(ck, ctx):
    dims = (32, 32, 512)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    ks, _ = ctx.make_shell_kernels(grid, [2.0], torch.float32)
    f = torch.zeros(dims, dtype=torch.float32, device=DEV)
    with pytest.raises(ck.ConkerError):   # field_b without its centre field
        ctx.convolve_contract(grid, f, f.clone(), ks, 3, centre_a=f.clone(), centre_b=None)
    with pytest.raises(ck.ConkerError):
        ctx.convolve_diag(grid, f, f.clone(), ks, 3, centre_a=f.clone(), centre_b=None)
