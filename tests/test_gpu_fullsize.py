"""Parity at full size: the survey-cap workload (512^3 grid, 30 shells, 800k + 32M
weighted tracers) in the configuration bench.py times, against the FP64 oracle
on sampled outputs it can afford: the histograms and alpha in full, the maps of
two shells at sampled cells (direct shell sums), and W_2, W_3 and W_4 for the
tuples among the sampled shells.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

SAMPLE = (0, 29)   # shell indices the oracle convolves (smallest and largest radius)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    w = synth.workload("cap512_ns800k_r30")
    data, rand = w.make()
    _say("catalogs", len(data), len(rand))
    D, wd, od = oc.histogram(data.pos, data.w, w.origin, w.cell, w.dims)
    R, wr, orr = oc.histogram(rand.pos, rand.w, w.origin, w.cell, w.dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    rc = [w.radii[m] / w.cell for m in SAMPLE]
    mN = oc.convolve_shells(N, rc)
    mR = oc.convolve_shells(R, rc)
    ref = {}
    for n in (2, 3, 4):
        tl = [tuple(SAMPLE[i] for i in t) for t in oc.radius_tuples(len(SAMPLE), n)]
        loc = [tuple(i for i in t) for t in oc.radius_tuples(len(SAMPLE), n)]
        ref[n] = (tl, oc.contract(N, mN, n, loc), oc.contract(R, mR, n, loc))
    _say("oracle done")
    return ck, w, data, rand, dict(alpha=alpha, N=N, R=R, wd=wd, wr=wr, out=(od, orr), ref=ref)


def _pick(W, ns, n, tuples):
    allt = oc.radius_tuples(ns, n)
    idx = {t: i for i, t in enumerate(allt)}
    return np.array([W[idx[t]] for t in tuples])


def _rel(got, ref):
    return float(np.abs(got - ref).max() / np.abs(ref).max())


def _rel_each(got, ref):
    """Tuple by tuple, for sums that are positive in every tuple (W_R)."""
    assert np.all(ref > 0)
    return float((np.abs(got - ref) / ref).max())


@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_cap512_full_size_sampled(cap, path):
    ck, w, data, rand, o = cap
    dev = "cuda:0"
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ctx = ck.Context(0)
    dt = torch.float64 if path == "fp64" else torch.float32
    prec = "f64" if path == "fp64" else "split_bf16"
    _say("full size", path)
    ks, sizes = ctx.make_shell_kernels(grid, w.radii, dt)
    assert sizes == [len(oc.shell_offsets(s / w.cell)) for s in w.radii]
    dpos, rpos = torch.from_numpy(data.pos).to(dev), torch.from_numpy(rand.pos).to(dev)
    dw, rw = torch.from_numpy(data.w).to(dev), torch.from_numpy(rand.w).to(dev)
    ns = len(w.radii)
    # one call for convolution and summation (float64: maps of carrying lines in
    # the context's workspace), then for float64 the separate calls, whose maps
    # are checked below
    runs = [(3, None), (2, None)] + ([(3, False)] if path == "fp64" else [])
    for n, fused in runs:
        _say("  n=%d fused=%s" % (n, fused))
        out = ck.npcf(ctx, grid, dpos, rpos, ks, n, dw, rw, precision=prec, dtype=dt, fused=fused)
        tl, rd, rr = o["ref"][n]
        gd = _pick(out["W_delta"].cpu().numpy(), ns, n, tl)
        gr = _pick(out["W_rand_raw"].cpu().numpy(), ns, n, tl)
        ed, er, ee = _rel(gd, rd), _rel(gr, rr), _rel_each(gr, rr)
        _say("  n=%d W_delta %.3e W_R %.3e (per tuple %.3e)" % (n, ed, er, ee))
        tol = 1e-12 if path == "fp64" else 1e-5
        assert ed <= tol and er <= tol and ee <= tol
        assert abs(out["alpha"].item() - o["alpha"]) <= 1e-13 * o["alpha"]
        b = out["bufs"]
        assert b["nout"].cpu().numpy().tolist() == list(o["out"]) == [0, 0]
    if path == "fp64":
        # maps of the separate path at sampled cells against direct shell sums
        maps_N = b["maps_N"]
        rng = np.random.default_rng(5)
        cells = np.stack([rng.integers(20, 492, 300), rng.integers(20, 492, 300), rng.integers(140, 372, 300)], 1)
        for m in SAMPLE:
            direct = oc.direct_shell_sum(o["N"], w.radii[m] / w.cell, cells)
            got = maps_N[m][cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy()
            assert np.abs(got - direct).max() <= 1e-11 * max(1.0, np.abs(direct).max())
    ctx.close()
    del ks
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["split_f16", "split_bf16"])
def test_cap512_full_size_n4(cap, prec):
    """Order 4 (4,960 tuples) on the survey cap: maps of the carrying lines in the
    workspace, then the matrix-core summation with split operands; the tuples
    among the two sampled shells against the oracle."""
    ck, w, data, rand, o = cap
    dev = "cuda:0"
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ctx = ck.Context(0)
    _say("full size n=4", prec)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, torch.float32)
    dpos, rpos = torch.from_numpy(data.pos).to(dev), torch.from_numpy(rand.pos).to(dev)
    dw, rw = torch.from_numpy(data.w).to(dev), torch.from_numpy(rand.w).to(dev)
    ns = len(w.radii)
    out = ck.npcf(ctx, grid, dpos, rpos, ks, 4, dw, rw, precision=prec, dtype=torch.float32)
    assert out["W_delta"].numel() == 4960
    tl, rd, rr = o["ref"][4]
    gd = _pick(out["W_delta"].cpu().numpy(), ns, 4, tl)
    gr = _pick(out["W_rand_raw"].cpu().numpy(), ns, 4, tl)
    ed, er, ee = _rel(gd, rd), _rel(gr, rr), _rel_each(gr, rr)
    _say("  n=4 W_delta %.3e W_R %.3e (per tuple %.3e)" % (ed, er, ee))
    assert ed <= 1e-5 and er <= 1e-5 and ee <= 1e-5
    ctx.close()
    del ks
    torch.cuda.empty_cache()


@pytest.mark.parametrize("order", [1, 5, 6, 0])
def test_cap512_fused_axis_orders(cap, order):
    """The fused pass on the survey cap with the axes transformed in the given
    order (1), in two fixed permutations (5: z, x, y; 6: z, y, x) and in the
    order chosen from the support (0): every one against the oracle."""
    ck, w, data, rand, o = cap
    dev = "cuda:0"
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ctx = ck.Context(0)
    ctx.set_tune(axis_order=order)
    _say("fused, axis order", order)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, torch.float32)
    dpos, rpos = torch.from_numpy(data.pos).to(dev), torch.from_numpy(rand.pos).to(dev)
    dw, rw = torch.from_numpy(data.w).to(dev), torch.from_numpy(rand.w).to(dev)
    ns = len(w.radii)
    for n in (3, 2):
        out = ck.npcf(ctx, grid, dpos, rpos, ks, n, dw, rw, precision="split_bf16", dtype=torch.float32)
        tl, rd, rr = o["ref"][n]
        ed = _rel(_pick(out["W_delta"].cpu().numpy(), ns, n, tl), rd)
        er = _rel(_pick(out["W_rand_raw"].cpu().numpy(), ns, n, tl), rr)
        _say("  n=%d W_delta %.3e W_R %.3e" % (n, ed, er))
        assert ed <= 1e-5 and er <= 1e-5
    ctx.close()
    del ks
    torch.cuda.empty_cache()
