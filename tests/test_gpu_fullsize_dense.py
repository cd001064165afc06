"""Parity at full size on the periodic boxes, against the FP64 oracle on the
outputs it can afford.

* box1280_ns300k_grid256_n5: 256^3 grid, 20 shells, 300k clustered points and
  3M randoms; order 5 (8,855 tuples) with split-bf16 and split-f16 operands and
  in float64: every tuple among four sampled shells (diagonal included) against
  oracle maps of those shells (Eq. ksin_delta at n = 5).
* box4096 on a 1024^3 grid of cell 4 with the catalog scaled to 1M + 10M
  points: the histograms compared in full (unit weights: exact), N, the maps
  of the smallest and largest shell (8 and 164 length units) at sampled cells
  against direct shell sums, and W_3 over those two shells with split-f16
  operands, the maps of one field at a time, as the 1024^3 workload runs.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
BOX_SAMPLE = (0, 6, 13, 19)       # shells of the 256^3 box the oracle convolves


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref):
    return float(np.abs(np.asarray(got) - np.asarray(ref)).max() / np.abs(ref).max())


def _rel_each(got, ref):
    assert np.all(ref > 0)
    return float((np.abs(np.asarray(got) - ref) / ref).max())


def _pick(W, ns, n, tuples):
    idx = {t: i for i, t in enumerate(oc.radius_tuples(ns, n))}
    return np.array([W[idx[t]] for t in tuples])


@pytest.fixture(scope="module")
def box256():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    w = synth.workload("box1280_ns300k_grid256_n5")
    data, rand = w.make()
    _say("box256 catalogs", len(data), len(rand))
    D, wd, _ = oc.histogram(data.pos, data.w, w.origin, w.cell, w.dims)
    R, wr, _ = oc.histogram(rand.pos, rand.w, w.origin, w.cell, w.dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    rc = [w.radii[m] / w.cell for m in BOX_SAMPLE]
    mN, mR = oc.convolve_shells(N, rc), oc.convolve_shells(R, rc)
    loc = oc.radius_tuples(len(BOX_SAMPLE), 5)
    tl = [tuple(BOX_SAMPLE[i] for i in t) for t in loc]
    ref = (tl, oc.contract(N, mN, 5, loc), oc.contract(R, mR, 5, loc))
    _say("box256 oracle done: %d tuples" % len(tl))
    return ck, w, data, rand, alpha, ref


@pytest.mark.parametrize("prec", ["split_bf16", "split_f16", "f64"])
def test_box256_n5_full_size(box256, prec):
    ck, w, data, rand, alpha, (tl, rd, rr) = box256
    dt = torch.float64 if prec == "f64" else torch.float32
    _say("box256 n=5", prec)
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ctx = ck.Context(0)
    ks, _ = ctx.make_shell_kernels(grid, w.radii, dt)
    out = ck.npcf(ctx, grid, torch.from_numpy(data.pos).to(DEV), torch.from_numpy(rand.pos).to(DEV), ks, 5,
                  precision=prec, dtype=dt)
    ns = len(w.radii)
    assert out["W_delta"].numel() == 8855
    gd = _pick(out["W_delta"].cpu().numpy(), ns, 5, tl)
    gr = _pick(out["W_rand_raw"].cpu().numpy(), ns, 5, tl)
    ed, er, ee = _rel(gd, rd), _rel(gr, rr), _rel_each(gr, rr)
    _say("  W_delta %.3e W_R %.3e (per tuple %.3e), %d tuples" % (ed, er, ee, len(tl)))
    tol = 1e-12 if prec == "f64" else 1e-5
    assert ed <= tol and er <= tol and ee <= tol
    assert abs(out["alpha"].item() - alpha) <= 1e-13 * alpha
    ctx.close()
    del ks
    torch.cuda.empty_cache()


def test_box1024_scaled_catalog(box256):
    """1024^3 cells (2^30): grids in full, two shells' maps at sampled cells and
    W_3 over those shells, split-f16, one field's maps at a time."""
    ck = box256[0]
    w = synth.workload("box4096_ns50m_grid1024")
    data, rand = w.make(scale=0.02)
    _say("box1024 catalogs", len(data), len(rand))
    grid = ck.Grid(w.dims, w.origin, w.cell)
    radii = [w.radii[0], w.radii[-1]]            # 8 and 164: shells of 2 and 41 cells
    ctx = ck.Context(0)
    dpos, rpos = torch.from_numpy(data.pos).to(DEV), torch.from_numpy(rand.pos).to(DEV)
    # ---- histograms in full (unit weights: integer counts, exact) -------------
    D_ref, wd, od = oc.histogram(data.pos, None, w.origin, w.cell, w.dims)
    R_ref, wr, orr = oc.histogram(rand.pos, None, w.origin, w.cell, w.dims)
    assert od == 0 and orr == 0
    for pos, ref, ws in ((dpos, D_ref, wd), (rpos, R_ref, wr)):
        g = torch.zeros(w.dims, dtype=torch.float32, device=DEV)
        s = torch.zeros(1, dtype=torch.float64, device=DEV)
        ctx.grid_assign(grid, pos, None, g, s)
        assert s.item() == ws
        assert np.array_equal(g.cpu().numpy(), ref.astype(np.float32))
        del g
    torch.cuda.empty_cache()
    _say("  histograms equal")
    # ---- the path the 1024^3 workload runs ------------------------------------
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
    out = ck.npcf(ctx, grid, dpos, rpos, ks, 3, precision="split_f16", dtype=torch.float32, field_at_a_time=True)
    gd, gr = out["W_delta"].cpu().numpy(), out["W_rand_raw"].cpu().numpy()
    N_gpu = out["bufs"]["N"]
    N_ref, alpha = oc.density_deviation(D_ref, R_ref, wd, wr)
    del D_ref
    assert abs(out["alpha"].item() - alpha) <= 1e-13 * alpha
    eN = float((N_gpu.cpu().numpy().astype(np.float64) - N_ref).__abs__().max())
    _say("  N: max |error| %.3e" % eN)
    assert eN <= 1e-6 * max(1.0, np.abs(N_ref).max())
    # maps of N from the GPU, at sampled cells
    maps = ctx.convolve_shells(grid, N_gpu, None, ks)[0]
    rng = np.random.default_rng(9)
    cells = rng.integers(0, 1024, size=(64, 3))
    got_maps = [maps[m][cells[:, 0], cells[:, 1], cells[:, 2]].cpu().numpy().astype(np.float64) for m in range(2)]
    del maps, out
    torch.cuda.empty_cache()
    # ---- oracle: one field's maps at a time -------------------------------------
    rc = [r / w.cell for r in radii]
    ref = {}
    for name, F in (("N", N_ref), ("R", R_ref)):
        mF = oc.convolve_shells(F, rc)
        ref[name] = oc.contract(F, mF, 3)
        if name == "N":
            for m in range(2):
                direct = oc.direct_shell_sum(F, rc[m], cells)
                scale = np.abs(mF[m]).max()
                e1 = np.abs(got_maps[m] - direct).max() / scale
                e2 = np.abs(direct - mF[m][cells[:, 0], cells[:, 1], cells[:, 2]]).max() / scale
                _say("  map %d at sampled cells: GPU %.3e, oracle FFT %.3e (of max |C|)" % (m, e1, e2))
                assert e1 <= 1e-5 and e2 <= 1e-12
        del mF
    ed, er, ee = _rel(gd, ref["N"]), _rel(gr, ref["R"]), _rel_each(gr, ref["R"])
    _say("  W_3 W_delta %.3e W_R %.3e (per tuple %.3e)" % (ed, er, ee))
    assert ed <= 1e-5 and er <= 1e-5 and ee <= 1e-5
    ctx.close()
    del ks
    torch.cuda.empty_cache()
