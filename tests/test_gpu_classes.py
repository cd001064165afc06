"""Size classes of a batch (conker_batch_plan with classes on): jobs on one grid
and kernel bank with their own buffers run stage by stage, one launch per
stage for the chunk.  Every class job must give what the same job gives when
the batch runs job by job, in the eager planning pass, an eager re-run and
HIP-graph replays, and one job per class is checked against the FP64 oracle
on the tuples among sampled shells.  Covered: two size classes (96^3 with a
radix-3 length, 128^3), split-bf16 and split-f16 summation, maps given by the
caller or kept in the class workspace, a 40-shell class (three summation
tiles), and a job whose grid buffer aliases a class member (it must run alone).
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
SAMPLE = (0, 7, 15)
MOCKS = ((96, 40_000), (128, 60_000), (96, 55_000), (128, 45_000), (96, 30_000))
CHECKED = (0, 1)                  # one job per class against the oracle

WIDE_CELL = 2.0
WIDE_RADII = tuple(4.0 + 1.4 * k for k in range(40))   # 40 shells, 2 .. 29.3 cells (the mocks' smallest: 2)
WIDE_SAMPLE = (0, 17, 39)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref):
    return float(np.abs(np.asarray(got) - np.asarray(ref)).max() / max(1e-300, np.abs(ref).max()))


def _oracle(mock, g, cell, radii, sample):
    d, r = mock
    dims = (g, g, g)
    D, wd, _ = oc.histogram(d.pos, d.w, (0.0, 0.0, 0.0), cell, dims)
    R, wr, _ = oc.histogram(r.pos, r.w, (0.0, 0.0, 0.0), cell, dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    rc = [radii[m] / cell for m in sample]
    mN, mR = oc.convolve_shells(N, rc), oc.convolve_shells(R, rc)
    loc = oc.radius_tuples(len(sample), 3)
    tl = [tuple(sample[i] for i in t) for t in loc]
    return alpha, tl, oc.contract(N, mN, 3, loc), oc.contract(R, mR, 3, loc)


def _pick(W, ns, tuples):
    idx = {t: i for i, t in enumerate(oc.radius_tuples(ns, 3))}
    return np.array([W[idx[t]] for t in tuples])


@pytest.fixture(scope="module")
def mocks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return [synth.mock_catalog(j, g, n, cell=CELL) for j, (g, n) in enumerate(MOCKS)]


@pytest.fixture(scope="module")
def oracle_classes(mocks):
    return {k: _oracle(mocks[k], MOCKS[k][0], CELL, RADII, SAMPLE) for k in CHECKED}


def _jobs(ck, ctx, sizes, cats, cell, radii, prec, stored, share_first=False):
    dev = "cuda:0"
    kspecs, jobs = {}, []
    for k, ((g, _), (d, r)) in enumerate(zip(sizes, cats)):
        grid = ck.Grid((g, g, g), (0.0, 0.0, 0.0), cell)
        if g not in kspecs:
            kspecs[g] = ctx.make_shell_kernels(grid, radii, torch.float32)[0]
        dp, rp = torch.from_numpy(d.pos).to(dev), torch.from_numpy(r.pos).to(dev)
        kw = {}
        if share_first and k == len(sizes) - 1:   # the last job maps into the first job's grids
            kw = dict(N=jobs[0].N, R=jobs[0].R)
        if stored:
            jobs.append(ck.make_job(grid, kspecs[g], 3, prec, dp, rp, fused=False, **kw))
        else:
            jobs.append(ck.make_job(grid, kspecs[g], 3, prec, dp, rp, fused=True, **kw))
    return jobs


def _outs(jobs):
    return [np.concatenate([j.W_delta.cpu().numpy(), j.W_rand.cpu().numpy(), j.xi.cpu().numpy(),
                            j.alpha.cpu().numpy(), j.wsum.cpu().numpy(), j.nout.cpu().numpy().astype(float)])
            for j in jobs]


def _run_both(ck, jobs, replays=3, **tune):
    """Outputs with classes (launch setting `tune`): plan, eager re-run, graph
    replays; then job by job with the defaults."""
    s = torch.cuda.Stream()
    ctx = ck.Context(0, stream=s)
    if tune:
        ctx.set_tune(**tune)
    torch.cuda.synchronize()
    ctx.batch_plan(jobs)
    layout = ctx.batch_layout()
    runs = [_outs(jobs)]
    for j in jobs:
        j.xi.zero_()
        j.W_delta.zero_()
    torch.cuda.synchronize()
    ctx.batch_run()
    ctx.synchronize()
    runs.append(_outs(jobs))
    ctx.batch_capture()
    for _ in range(replays):
        for j in jobs:   # eager work between replays: the graph must refill everything
            j.W_delta.fill_(7.0)
            j.W_rand.fill_(-3.0)
            j.xi.fill_(1.0)
            j.alpha.fill_(2.0)
            j.wsum.fill_(5.0)
        torch.cuda.synchronize()
        ctx.batch_launch()
        ctx.synchronize()
        runs.append(_outs(jobs))
    ctx.close()
    alone = ck.Context(0)
    alone.batch_classes(False)
    alone.batch_plan(jobs)
    assert alone.batch_layout() == [-1] * len(jobs)
    ref = _outs(jobs)
    alone.close()
    return layout, runs, ref


@pytest.mark.parametrize("prec,stored,radix", [(p, s, r) for p in ("split_bf16", "split_f16") for s in (False, True)
                                               for r in (0, 2)] + [("f32", False, 0), ("f32", False, 2)])
def test_classes_match_job_by_job_and_oracle(mocks, oracle_classes, prec, stored, radix):
    """bf16 and f32 without maps: the fused last pass and summation (f32 on
    v_mfma_f32_16x16x4f32); otherwise maps in the class workspace or the
    caller's buffers.  radix 2: the radix-16 schedule on the 128-cell axes."""
    import paper_2108_00015_amd as ck
    _say("classes", prec, "maps given" if stored else "maps in workspace", "radix", radix)
    ctx = ck.Context(0)
    jobs = _jobs(ck, ctx, MOCKS, mocks, CELL, RADII, prec, stored)
    layout, runs, ref = _run_both(ck, jobs, **({"radix": radix} if radix else {}))
    _say("  layout", layout)
    # one chunk per size class (the workspace bound holds these grids whole)
    assert layout[0] == layout[2] == layout[4] >= 0 and layout[1] == layout[3] >= 0 and layout[0] != layout[1]
    ns = len(RADII)
    nt = len(jobs[0].W_delta)
    for k in range(len(jobs)):
        for i, run in enumerate(runs):
            o = run[k]
            e = _rel(o[:3 * nt], ref[k][:3 * nt])
            assert e <= 1e-5, (k, i, e)
            assert np.array_equal(o[3 * nt + 1:], ref[k][3 * nt + 1:]), k   # weight sums, rejected counts
            assert abs(o[3 * nt] - ref[k][3 * nt]) <= 1e-13 * ref[k][3 * nt]
    for k in CHECKED:
        alpha, tl, rd, rr = oracle_classes[k]
        got = runs[-1][k]
        ed, er = _rel(_pick(got[:nt], ns, tl), rd), _rel(_pick(got[nt:2 * nt], ns, tl), rr)
        _say("  oracle job %d (%d^3): W_delta %.3e W_R %.3e" % (k, MOCKS[k][0], ed, er))
        assert ed <= 1e-5 and er <= 1e-5
        assert abs(got[3 * nt] - alpha) <= 1e-13 * alpha
    ctx.close()


def test_classes_forty_shells_and_aliasing():
    """A class of three 64^3 jobs with 40 shells (the summation's three-tile
    form), plus a fourth job whose grids are the first job's: it runs alone,
    after the class, and every job still matches the job-by-job batch; the
    first job against the oracle at sampled shells."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    sizes = ((64, 20_000), (64, 25_000), (64, 15_000), (64, 18_000))
    cats = [synth.mock_catalog(20 + j, g, n, cell=WIDE_CELL) for j, (g, n) in enumerate(sizes)]
    ctx = ck.Context(0)
    jobs = _jobs(ck, ctx, sizes, cats, WIDE_CELL, WIDE_RADII, "split_bf16", False, share_first=True)
    layout, runs, ref = _run_both(ck, jobs, replays=2)
    _say("40 shells, layout", layout)
    assert layout[0] == layout[1] == layout[2] >= 0 and layout[3] == -1
    nt = len(jobs[0].W_delta)
    for k in range(len(jobs)):
        for i, run in enumerate(runs):
            e = _rel(run[k][:3 * nt], ref[k][:3 * nt])
            assert e <= 1e-5, (k, i, e)
    alpha, tl, rd, rr = _oracle(cats[0], 64, WIDE_CELL, WIDE_RADII, WIDE_SAMPLE)
    got = runs[-1][0]
    ed = _rel(_pick(got[:nt], len(WIDE_RADII), tl), rd)
    er = _rel(_pick(got[nt:2 * nt], len(WIDE_RADII), tl), rr)
    _say("  oracle job 0: W_delta %.3e W_R %.3e" % (ed, er))
    _say("  per tuple W_delta", np.abs(_pick(got[:nt], len(WIDE_RADII), tl) - rd) / np.abs(rd).max())
    assert ed <= 1e-5 and er <= 1e-5
    ctx.close()


def test_mock_batch_full_size_as_benched():
    """The 64-mock batch exactly as bench.py times it (grids 96..256 cells,
    50k..400k clustered points + 10x randoms, 16 shells, split-bf16, per-job
    grids, no map buffers: size classes with the fused last pass and
    summation, captured as one graph): one mock of each grid size against the
    oracle on the tuples among three sampled shells, and alpha; the graph
    replay against the eager planning pass for every mock."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as ck
    sizes = synth.mock_sizes(64, 400)
    cats = [synth.mock_catalog(j, g, n) for j, (g, n) in enumerate(sizes)]
    dev = "cuda:0"
    s = torch.cuda.Stream()
    ctx = ck.Context(0, stream=s)
    kspecs, jobs = {}, []
    for (g, _), (d, r) in zip(sizes, cats):
        grid = ck.Grid((g, g, g), (0.0, 0.0, 0.0), CELL)
        if g not in kspecs:
            kspecs[g] = ctx.make_shell_kernels(grid, RADII, torch.float32)[0]
        jobs.append(ck.make_job(grid, kspecs[g], 3, "split_bf16", torch.from_numpy(d.pos).to(dev),
                                torch.from_numpy(r.pos).to(dev), fused=True))
    torch.cuda.synchronize()
    ctx.batch_plan(jobs)
    layout = ctx.batch_layout()
    _say("full mock batch, chunks", sorted(set(layout)), "alone", layout.count(-1))
    assert min(layout) >= 0   # every mock runs in a size class
    first = _outs(jobs)
    ctx.batch_capture()
    for j in jobs:
        j.W_delta.fill_(7.0)
        j.W_rand.fill_(-3.0)
    torch.cuda.synchronize()
    ctx.batch_launch()
    ctx.synchronize()
    again = _outs(jobs)
    nt = len(jobs[0].W_delta)
    for k in range(len(jobs)):
        assert _rel(again[k][:3 * nt], first[k][:3 * nt]) <= 1e-5, k
    ns = len(RADII)
    for g in sorted({g for g, _ in sizes}):
        k = next(i for i, (gg, _) in enumerate(sizes) if gg == g)
        alpha, tl, rd, rr = _oracle(cats[k], g, CELL, RADII, SAMPLE)
        got = again[k]
        ed, er = _rel(_pick(got[:nt], ns, tl), rd), _rel(_pick(got[nt:2 * nt], ns, tl), rr)
        _say("  mock %d (%d^3): W_delta %.3e W_R %.3e" % (k, g, ed, er))
        assert ed <= 1e-5 and er <= 1e-5
        assert abs(got[3 * nt] - alpha) <= 1e-13 * alpha
    ctx.close()
