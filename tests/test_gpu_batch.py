"""Batches of independent mocks through conker_batch_*: the eager planning pass,
eager re-runs and HIP-graph replays agree with each other and with the FP64
oracle (Eq. ksi3combined is then a sum over jobs).  Grids of 96, 128, 192 and
256 cells per side (every size class of the mock workload, radix-3 FFT lengths
beside the powers of two) with 50k-400k clustered points and ten times as many
randoms; one mock of each size class is checked against the oracle.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conker as oc  # noqa: E402
import synth  # noqa: E402

pytestmark = pytest.mark.gpu

CELL = 5.0
RADII = synth.MOCK_RADII          # 16 shells, 10 .. 85
SAMPLE = (0, 7, 15)               # shells the oracle convolves
MOCKS = ((96, 50_000), (128, 120_000), (192, 250_000), (96, 80_000), (256, 400_000))
CHECKED = (0, 1, 2, 4)            # one mock of each size class against the oracle


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref):
    return float(np.abs(np.asarray(got) - np.asarray(ref)).max() / max(1e-300, np.abs(ref).max()))


@pytest.fixture(scope="module")
def mocks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [synth.mock_catalog(j, g, n, cell=CELL) for j, (g, n) in enumerate(MOCKS)]


def _oracle_mock(mock, g):
    """FP64 oracle for one mock: alpha, and W_n over the tuples of SAMPLE (n = 2, 3)."""
    d, r = mock
    dims = (g, g, g)
    D, wd, _ = oc.histogram(d.pos, d.w, (0.0, 0.0, 0.0), CELL, dims)
    R, wr, _ = oc.histogram(r.pos, r.w, (0.0, 0.0, 0.0), CELL, dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    rc = [RADII[m] / CELL for m in SAMPLE]
    mN, mR = oc.convolve_shells(N, rc), oc.convolve_shells(R, rc)
    ref = {}
    for n in (2, 3):
        loc = oc.radius_tuples(len(SAMPLE), n)
        tl = [tuple(SAMPLE[i] for i in t) for t in loc]
        ref[n] = (tl, oc.contract(N, mN, n, loc), oc.contract(R, mR, n, loc))
    return alpha, ref


@pytest.fixture(scope="module")
def oracle_classes(mocks):
    """The oracle of one mock per size class: {job index: (alpha, ref)}."""
    return {k: _oracle_mock(mocks[k], MOCKS[k][0]) for k in CHECKED}


def _pick(W, n, tuples):
    idx = {t: i for i, t in enumerate(oc.radius_tuples(len(RADII), n))}
    return np.array([W[idx[t]] for t in tuples])


def _build(ck, ctx, mocks, n, dtype, prec, stored=True):
    dev = "cuda:0"
    kspecs = {}
    gmax = max(g for g, _ in MOCKS)
    ncmax = gmax ** 3
    N = torch.empty(ncmax, dtype=dtype, device=dev)
    R = torch.empty(ncmax, dtype=dtype, device=dev)
    mN = torch.empty(len(RADII) * ncmax, dtype=dtype, device=dev)
    mR = torch.empty(len(RADII) * ncmax, dtype=dtype, device=dev)
    jobs = []
    for (g, _), (d, r) in zip(MOCKS, mocks):
        grid = ck.Grid((g, g, g), (0.0, 0.0, 0.0), CELL)
        if g not in kspecs:
            kspecs[g] = ctx.make_shell_kernels(grid, RADII, dtype)[0]
        dp = torch.from_numpy(d.pos).to(dev)
        rp = torch.from_numpy(r.pos).to(dev)
        if stored:
            jobs.append(ck.make_job(grid, kspecs[g], n, prec, dp, rp, N=N, R=R, maps_N=mN, maps_R=mR, fused=False))
        else:   # conker_convolve_contract: maps of carrying lines in the context's workspace
            jobs.append(ck.make_job(grid, kspecs[g], n, prec, dp, rp, N=N, R=R, fused=True))
    return jobs


def _outs(jobs):
    return [np.concatenate([j.W_delta.cpu().numpy(), j.W_rand.cpu().numpy(), j.xi.cpu().numpy(),
                            j.alpha.cpu().numpy()]) for j in jobs]


@pytest.mark.parametrize("maps", ["stored", "workspace"])
@pytest.mark.parametrize("path", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [3, 2])
def test_batch_eager_graph_oracle(mocks, oracle_classes, path, n, maps):
    import paper_2108_00015_amd as ck
    dtype = torch.float64 if path == "fp64" else torch.float32
    prec = "f64" if path == "fp64" else "split_bf16"
    tol_self = 1e-12 if path == "fp64" else 1e-5     # atomics reorder the scatter sums
    tol_ref = 1e-12 if path == "fp64" else 1e-5
    _say("batch", path, "n=%d" % n, maps, [g for g, _ in MOCKS])
    s = torch.cuda.Stream()
    ctx = ck.Context(0, stream=s)
    jobs = _build(ck, ctx, mocks, n, dtype, prec, stored=maps == "stored")
    assert all((j.maps_N is None) == (maps == "workspace") for j in jobs)
    torch.cuda.synchronize()
    ctx.batch_plan(jobs)
    first = _outs(jobs)
    for j in jobs:
        j.xi.zero_()
    torch.cuda.synchronize()
    ctx.batch_run()
    ctx.synchronize()
    again = _outs(jobs)
    ctx.batch_capture()
    graphs = []
    for rep in range(3):
        for j in jobs:               # eager work between replays; the graph must refill everything
            j.W_delta.fill_(7.0)
            j.W_rand.fill_(-3.0)
            j.xi.fill_(1.0)
        torch.cuda.synchronize()
        ctx.batch_launch()
        ctx.synchronize()
        graphs.append(_outs(jobs))
    for k in range(len(jobs)):
        for o in [again[k]] + [gr[k] for gr in graphs]:
            assert _rel(o, first[k]) <= tol_self, (k, _rel(o, first[k]))
    # oracle on one mock per size class, from the last graph replay
    for k in CHECKED:
        alpha, ref = oracle_classes[k]
        tl, rd, rr = ref[n]
        jk = jobs[k]
        nt = len(jk.W_delta)
        gd = _pick(graphs[-1][k][:nt], n, tl)
        gr_ = _pick(graphs[-1][k][nt:2 * nt], n, tl)
        ed, er = _rel(gd, rd), _rel(gr_, rr)
        _say("  oracle mock %d (%d^3): W_delta %.3e W_R %.3e" % (k, MOCKS[k][0], ed, er))
        assert ed <= tol_ref and er <= tol_ref, k
        assert abs(jk.alpha.item() - alpha) <= 1e-13 * alpha
    ctx.close()


def test_batch_rejects_bad_jobs(mocks):
    import paper_2108_00015_amd as ck
    ctx = ck.Context(0, stream=torch.cuda.Stream())
    jobs = _build(ck, ctx, mocks[:1], 3, torch.float32, "split_bf16")
    jobs[0].n = 6
    with pytest.raises(ck.ConkerError):
        ctx.batch_plan(jobs)
    jobs[0].n = 3
    jobs[0].maps_N = None           # maps_R still given
    with pytest.raises(ck.ConkerError):
        ctx.batch_plan(jobs)
    with pytest.raises(ck.ConkerError):
        ctx.batch_launch()
    ctx.close()


def test_batch_fused_jobs_graph_replay():
    """Jobs on a grid with 512-cell z lines take the fused pass (line masks,
    list-driven transforms); graph replays match the eager pass and the oracle.
    The data are clustered: for unclustered data W_delta is shot noise far
    below the size of its terms, and its float32 error relative to max |W_delta|
    measures that cancellation rather than the path."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    DEV = "cuda:0"
    dims, cell = (32, 64, 512), 1.0
    radii = [1.0, 2.0, 3.5, 5.0, 8.0, 12.0]
    cats = []
    for j in range(3):
        d = synth.neyman_scott_box(4000 + 1000 * j, 40, 1.5, 0.0, 30.0, seed=500 + j)
        r = synth.uniform_box(40000, 0.0, 30.0, seed=700 + j)
        cats.append((d, r))
    s = torch.cuda.Stream()
    ctx = ck.Context(0, stream=s)
    grid = ck.Grid(dims, (0, 0, 0), cell)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
    jobs = [ck.make_job(grid, ks, 3, "split_bf16", torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV))
            for d, r in cats]
    assert all(j.maps_N is None for j in jobs)      # fused
    torch.cuda.synchronize()
    ctx.batch_plan(jobs)
    first = _outs(jobs)
    ctx.batch_capture()
    for rep in range(3):
        for j in jobs:
            j.W_delta.fill_(5.0)
            j.xi.fill_(0.0)
        torch.cuda.synchronize()
        ctx.batch_launch()
        ctx.synchronize()
        for k, o in enumerate(_outs(jobs)):
            assert _rel(o, first[k]) <= 1e-5, (rep, k)
    for k, (d, r) in enumerate(cats):
        ref = oc.npcf(d, r, dims, (0, 0, 0), cell, radii, 3)
        assert _rel(jobs[k].W_delta.cpu().numpy(), ref["W_delta"]) <= 1e-5
        assert _rel(jobs[k].W_rand.cpu().numpy(), ref["W_rand_raw"]) <= 1e-5
    ctx.close()


def test_batch_axis_order_under_graph_capture():
    """Fused jobs on a cubic 512^3 grid with cone-shaped support: the axis
    order is chosen on the device inside the captured graph.  Replays match
    the eager pass, and both match the same jobs in the given axis order (the
    order only changes the summation order; float32 bar 1e-5)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    DEV = "cuda:0"
    L = 512
    radii = [2.0, 3.5, 5.0, 8.0, 11.0, 14.0, 17.0, 20.0]   # enough radii for the copies to pay
    cats = []
    for j in range(2):
        rng = np.random.default_rng(900 + j)
        # points in a cone along z: few z-slabs, most x- and y-slabs
        m = 60_000 + 20_000 * j
        z = rng.uniform(250.0, 330.0, size=m)
        rr = 0.6 * z * np.sqrt(rng.uniform(0, 1, size=m))
        ph = rng.uniform(0, 2 * np.pi, size=m)
        pts = np.stack([256 + rr * np.cos(ph) * 0.6, 256 + rr * np.sin(ph) * 0.6, z], 1).astype(np.float32)
        cats.append((pts[: m // 10], pts))
    grid = ck.Grid((L, L, L), (0, 0, 0), 1.0)

    def run(order):
        s = torch.cuda.Stream()
        ctx = ck.Context(0, stream=s)
        ctx.set_tune(axis_order=order)
        ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
        jobs = [ck.make_job(grid, ks, 3, "split_bf16", torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV))
                for d, r in cats]
        assert all(j.maps_N is None for j in jobs)
        torch.cuda.synchronize()
        ctx.batch_plan(jobs)
        used = ctx.axis_order_used()
        first = _outs(jobs)
        ctx.batch_capture()
        reps = []
        for rep in range(3):
            for j in jobs:
                j.W_delta.fill_(5.0)
                j.xi.fill_(0.0)
            torch.cuda.synchronize()
            ctx.batch_launch()
            ctx.synchronize()
            reps.append(_outs(jobs))
        ctx.close()
        return used, first, reps

    used, first, reps = run(0)
    assert used in (5, 6), used
    for r in reps:
        for k in range(len(cats)):
            assert np.array_equal(r[k], first[k]), k        # the graph repeats the eager arithmetic
    used1, given, _ = run(1)
    assert used1 == 1
    for k in range(len(cats)):
        assert _rel(first[k], given[k]) <= 1e-5, (k, _rel(first[k], given[k]))


def test_batch_graph_dropped_when_workspace_grows():
    """A captured batch records the context's workspace addresses.  An eager
    call that makes the workspace grow (here a larger grid) frees those
    buffers, so the captured batch is dropped with them: launching it then
    reports an error instead of replaying on freed memory, and a new capture
    runs again."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    DEV = "cuda:0"
    dims, cell = (32, 32, 512), 1.0
    radii = [1.0, 2.0, 3.5]
    d = synth.neyman_scott_box(3000, 30, 1.5, 0.0, 30.0, seed=520)
    r = synth.uniform_box(30000, 0.0, 30.0, seed=720)
    ctx = ck.Context(0, stream=torch.cuda.Stream())
    grid = ck.Grid(dims, (0, 0, 0), cell)
    ks, _ = ctx.make_shell_kernels(grid, radii, torch.float32)
    jobs = [ck.make_job(grid, ks, 3, "split_bf16", torch.from_numpy(d).to(DEV), torch.from_numpy(r).to(DEV))]
    torch.cuda.synchronize()
    ctx.batch_plan(jobs)
    first = _outs(jobs)
    ctx.batch_capture()
    ctx.batch_launch()
    ctx.synchronize()
    # an eager call on a grid four times larger grows the spectrum buffers
    big = ck.Grid((64, 64, 512), (0, 0, 0), cell)
    ksb, _ = ctx.make_shell_kernels(big, radii, torch.float32)
    f = torch.zeros(big.dims, dtype=torch.float32, device=DEV)
    f[10, 10, 10] = 1.0
    ctx.convolve_contract(big, f, f.clone(), ksb, 3, "split_bf16")
    ctx.synchronize()
    with pytest.raises(ck.ConkerError) as e:
        ctx.batch_launch()
    assert "no captured batch" in str(e.value)
    ctx.batch_capture()
    for j in jobs:
        j.W_delta.fill_(5.0)
    torch.cuda.synchronize()
    ctx.batch_launch()
    ctx.synchronize()
    for k, o in enumerate(_outs(jobs)):
        assert _rel(o, first[k]) <= 1e-5
    ctx.close()
