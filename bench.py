"""Throughput of the ConKer hot path on one MI355X.

One step = mapping (NGP scatter of data and randoms, N = D - alpha R) ->
convolution of N and R_raw with every shell kernel (2 * N_s shell
convolutions) -> n-point summation of both fields -> float64 ratio, on a
synthetic survey-shaped catalog already resident in GPU memory.  The shell
kernel spectra are built once per grid and radius set, outside the timed
region.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  `value` is shell convolutions completed per second of
whole-step time on the mixed-precision path (float32 FFTs, split-bf16 matrix
core summation); the float64 path is timed beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "s to W_3 at 512³ grid, 30 radii (mixed-prec vs FP64 GPU); shell-convs/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(kind, n_launch_units, nc, ns, kel, n_data, n_rand, weighted, esize, batch, fx=1.0, fl=1.0,
                 pruned_fwd=False):
    """Algorithmic HBM bytes of all launches of one kind in one step.

    esize = bytes of one real value (4 or 8); complex = 2 * esize.  When the maps
    are only summed, the inverse passes produce their outputs on the z-lines that
    carry field (fraction fl of all lines, in a fraction fx of the x-slabs):
    the x pass writes fx of its output, the y pass reads fx and writes fl, the
    z pass reads fl.  With the axes permuted (axis_order), x, y and z are the
    axes of the permuted grid: fx is the fraction of its first-axis slabs and fl
    that of lines along its last axis.  With pruned_fwd (auto-correlations in
    one call: the fields are zero off their own support) the forward passes are
    pruned the same way: the z pass reads and writes carrying lines only, the y
    pass reads them and writes the slabs holding them, the x pass reads those
    slabs and writes every cell.
    """
    c = 2 * esize
    gz, gy_in, gy_out, gx_in = (fl, fl, fx, fx) if pruned_fwd else (1.0, 1.0, 1.0, 1.0)
    if kind == "fft_fwd_z":       # two real fields in, one complex field out
        return gz * (2 * nc * esize + nc * c)
    if kind == "fft_fwd_y":
        return (gy_in + gy_out) * nc * c
    if kind == "fft_fwd_x":
        return (gx_in + 1.0) * nc * c
    if kind == "pack_scale":      # both fields read once for their sums of squares
        return 2 * nc * esize
    if kind == "fft_inv_x_mul":   # spectrum read once per batch, kernel octant + output per radius
        n_batches = math.ceil(ns / batch)
        return n_batches * nc * c + ns * (kel * esize + fx * nc * c)
    if kind == "fft_inv_y":
        return ns * (fx + fl) * nc * c
    if kind == "support":         # both fields read once
        return 2 * nc * esize
    if kind == "axis_order":      # both fields read for the projections, then read and written permuted
        return 6 * nc * esize
    if kind == "diag_zinv":
        return ns * fl * nc * c + 2 * fl * nc * esize
    if kind == "fft_inv_z":       # complex in, two real maps out (carrying lines, or every line)
        return ns * fl * (nc * c + 2 * nc * esize)
    if kind == "scatter":         # positions (+ weights) in, one grid value read-modify-write per point
        per = 12 + (4 if weighted else 0) + 2 * esize
        return (n_data + n_rand) * per
    if kind == "form_delta":
        return 3 * nc * esize
    if kind == "fused_zinv_contract":   # every radius's spectrum and both fields, on carrying lines
        return ns * fl * nc * c + 2 * fl * nc * esize
    return None


# rocprofv3 counter runs of the dominant kernel (FETCH_SIZE, WRITE_SIZE per
# dispatch, KiB) are committed under profiles/ together with a hash of the
# sources the kernel is built from; the figure is used only while they match.
TRAFFIC_SOURCES = ("paper_2108_00015_amd/csrc/fft.hip", "paper_2108_00015_amd/csrc/fft_math.h",
                   "paper_2108_00015_amd/csrc/common.h", "paper_2108_00015_amd/csrc/fused.hip",
                   "paper_2108_00015_amd/csrc/order.hip", "paper_2108_00015_amd/csrc/support.hip",
                   "paper_2108_00015_amd/csrc/split3.h", "paper_2108_00015_amd/csrc/batch.hip")


def source_hashes(paths=TRAFFIC_SOURCES):
    import hashlib
    out = {}
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            out[rel] = hashlib.sha256(f.read()).hexdigest()
    return out


def measured_traffic(kind, workload, n):
    """HBM bytes per launch of `kind` from the committed counter summary, or None
    when there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s_n%d.json" % (kind, workload, n))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("sources") != source_hashes(tuple(t.get("sources", {}).keys()) or TRAFFIC_SOURCES):
        return None
    return (t["fetch_kib_per_dispatch"] * t["fetch_factor"] + t["write_kib_per_dispatch"] * t["write_factor"]) * 1024.0


MFMA_PEAK_TFLOPS = {"split_bf16": 2500.0, "split_f16": 2500.0, "f32": 157.3, "f64": 78.6}
TERM_PRODUCTS = {"split_bf16": 6, "split_f16": 3, "f32": 1, "f64": 1}


def summation_tiles(ns, n, ts=32):
    """32 x 32 output tiles the matrix-core summation issues for order n (row items
    F C_a or F C_a C_b, column items C_b or C_c C_d, as in the library's plan:
    row pairs ordered by their larger radius, column pairs lexicographically)."""
    singles = [(a,) for a in range(ns)]
    pairs = [(a, b) for a in range(ns) for b in range(a, ns)]
    rows_by_b = sorted(pairs, key=lambda p: (p[1], p[0]))
    if n == 3:
        left, right = singles, singles
    elif n == 4:
        left, right = rows_by_b, singles
    else:
        left, right = rows_by_b, pairs
    li = {t: i for i, t in enumerate(left)}
    ri = {t: i for i, t in enumerate(right)}
    import itertools
    tiles = set()
    for t in itertools.combinations_with_replacement(range(ns), n - 1):
        if n == 3:
            a, b = (t[0],), (t[1],)
        elif n == 4:
            a, b = (t[0], t[1]), (t[2],)
        else:
            a, b = (t[0], t[1]), (t[2], t[3])
        tiles.add((li[a] // ts, ri[b] // ts))
    return len(tiles)


def comb_tuples(ns, n):
    return math.comb(ns + n - 2, n - 1)


def roofline_of(stages, n, prec, workload, time_key="ms_per_step", note=None):
    """The roofline entry of the dominant kernel (largest time per step).

    stages: {kind: {time_key, avg_launch_ms, and gbs + bytes_per_launch where
    the byte model applies, mfma_issued_tflops for the separate summation}}.
    Orders 4 and 5 are bound by the matrix cores when the separate summation
    dominates: issued matrix flops (every split product counted) per launch
    against the dense peak of the operand type, the unsplit count beside them.
    Otherwise the kernel is priced on HBM by its algorithmic bytes per launch,
    with the committed counter traffic when it matches the sources.
    """
    if not stages:
        return None
    kind, ent = max(stages.items(), key=lambda kv: kv[1][time_key])
    if kind == "contract_mm" and n >= 4 and "mfma_issued_tflops" in ent:
        issued = ent["mfma_issued_tflops"] * 1e12 * ent["avg_launch_ms"] * 1e-3
        peak = MFMA_PEAK_TFLOPS[prec]
        return dict(bound="mfma", kernel=kind, achieved=ent["mfma_issued_tflops"], peak=peak, unit="TFLOP/s",
                    frac=round(ent["mfma_issued_tflops"] / peak, 4), traffic=None,
                    flops_per_launch=issued, algorithmic_flops_per_launch=issued / TERM_PRODUCTS[prec],
                    term_products=TERM_PRODUCTS[prec], avg_launch_ms=ent["avg_launch_ms"])
    if "gbs" not in ent:
        return None
    ach = ent["bytes_per_launch"] / (ent["avg_launch_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(kind, workload, n)
    roof = dict(bound="hbm", kernel=kind, achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=round(ach / HBM_PEAK_GBS, 4),
                traffic=(int(round(traffic)) if traffic is not None else None), traffic_unit="bytes/launch",
                bytes_per_launch=ent["bytes_per_launch"], avg_launch_ms=ent["avg_launch_ms"])
    if note:
        roof["note"] = note
    return roof


def stages_use_fused(prof):
    return "fused_zinv_contract" in prof


AXIS_ORDERS = {1: (0, 1, 2), 2: (0, 2, 1), 3: (1, 0, 2), 4: (1, 2, 0), 5: (2, 0, 1), 6: (2, 1, 0)}


def support_fractions(w, data, rand, order=1):
    """For the axes transformed in `order` (1..6, new axis k = old axis
    AXIS_ORDERS[order][k]): the fraction of first-axis slabs, of lines along
    the last axis and of 64-cell blocks of the permuted grid (runs of 64 cells
    along that axis, the unit the summation skips) holding at least one
    catalog point (where N or R_raw can be non-zero)."""
    dims = np.asarray(w.dims)
    occ = np.zeros(tuple(int(d) for d in dims), dtype=bool)
    o = np.asarray(w.origin, dtype=np.float64)
    for cat in (data, rand):
        for s in range(0, len(cat), 1 << 24):
            c = np.floor((cat.pos[s:s + (1 << 24)].astype(np.float64) - o) / w.cell).astype(np.int64)
            ok = np.all((c >= 0) & (c < dims), axis=1)
            occ[c[ok, 0], c[ok, 1], c[ok, 2]] = True
    first, last = AXIS_ORDERS[order][0], AXIS_ORDERS[order][2]
    others = tuple(a for a in range(3) if a != first)
    fx = float(occ.any(axis=others).mean())
    fl = float(occ.any(axis=last).mean())
    lines = np.moveaxis(occ, last, -1)
    n_last = lines.shape[-1]
    if n_last % 64 == 0:
        fb = float(lines.reshape(-1, n_last // 64, 64).any(axis=2).mean())
    else:   # blocks straddle lines: count them on the flat permuted grid
        flat = np.moveaxis(occ, AXIS_ORDERS[order], (0, 1, 2)).reshape(-1)
        pad = (-flat.size) % 64
        fb = float(np.concatenate([flat, np.zeros(pad, bool)]).reshape(-1, 64).any(axis=1).mean())
    return fx, fl, fb


def cpu_baseline(w, data, rand, n, sample_radii=1):
    """The FP64 oracle on a bounded sample, extrapolated to one full step.

    Sample: full mapping of both catalogs; convolution of both fields with the
    first `sample_radii` shells; summation of the tuples among those shells.
    The full-step time is mapping + (N_s / k) x convolution + (T / T_k) x summation.
    """
    from oracle import conker as oc
    ns = len(w.radii)
    t0 = time.perf_counter()
    D, wd, _ = oc.histogram(data.pos, data.w, w.origin, w.cell, w.dims)
    R, wr, _ = oc.histogram(rand.pos, rand.w, w.origin, w.cell, w.dims)
    N, alpha = oc.density_deviation(D, R, wd, wr)
    t1 = time.perf_counter()
    rc = [s / w.cell for s in w.radii[:sample_radii]]
    mN = oc.convolve_shells(N, rc)
    mR = oc.convolve_shells(R, rc)
    t2 = time.perf_counter()
    oc.contract(N, mN, n)
    oc.contract(R, mR, n)
    t3 = time.perf_counter()
    k = sample_radii
    full = (t1 - t0) + (ns / k) * (t2 - t1) + (oc.num_tuples(ns, n) / oc.num_tuples(k, n)) * (t3 - t2)
    return dict(value=2 * ns / full, unit="shell-convs/s", cores=len(os.sched_getaffinity(0)), kind="oracle",
                sample=("full mapping of both catalogs, convolution of both fields with %d of %d shells, "
                        "summation (n=%d) over the %d tuples of those shells; extrapolated to all %d shells "
                        "and %d tuples" % (k, ns, n, oc.num_tuples(k, n), ns, oc.num_tuples(ns, n))),
                sample_seconds=t3 - t0, extrapolated_step_seconds=full,
                stage_seconds=dict(mapping=t1 - t0, convolution=t2 - t1, summation=t3 - t2))


def run_path(ck, torch, ctx, grid, w, dpos, dw, rpos, rw, n, dtype, prec, steps, warmup, profile,
             mode="npcf", field_at_a_time=False):
    ks, _ = ctx.make_shell_kernels(grid, w.radii, dtype)
    torch.cuda.synchronize()
    bufs = {}

    def step():
        if mode == "diag":
            out = ck.npcf_diag(ctx, grid, dpos, rpos, ks, n, dw, rw, dtype=dtype, allow_outside=True)
            return dict(out, W_delta=out["W_delta"].reshape(-1), W_rand_raw=out["W_rand_raw"].reshape(-1))
        if mode == "pair2":
            return ck.npcf_pair2(ctx, grid, dpos, rpos, ks, dw, rw, dtype=dtype, allow_outside=True)
        return ck.npcf(ctx, grid, dpos, rpos, ks, n, dw, rw, precision=prec, dtype=dtype, bufs=bufs,
                       field_at_a_time=field_at_a_time, allow_outside=True)

    for _ in range(warmup):
        out = step()
    torch.cuda.synchronize()
    if profile:
        ctx.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        out = step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    prof = ctx.profile_read() if profile else {}
    # every tracer of the workload lies inside the grid (checked once, outside the timed steps)
    outside = [int(v) for v in out["n_outside"].cpu().tolist()]
    if any(outside):
        raise RuntimeError("tracers outside the grid: %s" % outside)
    if profile:
        ctx.profile(False)
    res = dict(ms=ms, xi=out["xi"].cpu().numpy(), Wd=out["W_delta"].cpu().numpy(),
               Wr=out["W_rand_raw"].cpu().numpy(), alpha=float(out["alpha"].item()), prof=prof,
               workspace=ctx.workspace_bytes(), axis_order=ctx.axis_order_used() or 1)
    del bufs, ks, out
    torch.cuda.empty_cache()
    return res


MOCKS_NAME = "mocks64_periodic_grid96-256_r16"


def mock_stage_bytes(kind, sizes, ns, npts, nb=8):
    """Algorithmic HBM bytes of one kind of launch over a whole mock batch run as
    size classes (float32 grids, every line carries field: periodic boxes; nb
    radii transformed per batch)."""
    tot = 0.0
    for (g, _), n in zip(sizes, npts):
        nc = g ** 3
        kel = (g // 2 + 1) ** 3
        if kind == "contract_mm":     # field and maps of both fields, every block
            b = 2 * (ns + 1) * nc * 4
        elif kind == "scatter":       # zeroing both grids, positions in, one grid RMW per point
            b = 2 * nc * 4 + n * (12 + 8)
        elif kind == "contract_reduce":
            b = None
        else:
            b = kernel_bytes(kind, 1, nc, ns, kel, n, 0, False, 4, nb)
        if b is None:
            return None
        tot += b
    return tot


def mocks_cpu_baseline(sizes, cats, radii, n, k=16):
    """The FP64 oracle on one mock of each grid size (mapping, k shells,
    summation over the tuples of those shells), extrapolated to every shell and
    tuple and to the batch's count of mocks of that size."""
    from oracle import conker as oc
    ns = len(radii)
    total, parts = 0.0, {}
    t_all = time.perf_counter()
    for g in sorted({g for g, _ in sizes}):
        d, r = cats[next(i for i, (gg, _) in enumerate(sizes) if gg == g)]
        dims = (g, g, g)
        t0 = time.perf_counter()
        D, wd, _ = oc.histogram(d.pos, d.w, (0.0, 0.0, 0.0), 5.0, dims)
        R, wr, _ = oc.histogram(r.pos, r.w, (0.0, 0.0, 0.0), 5.0, dims)
        N, _ = oc.density_deviation(D, R, wd, wr)
        t1 = time.perf_counter()
        rc = [s / 5.0 for s in radii[:k]]
        mN, mR = oc.convolve_shells(N, rc), oc.convolve_shells(R, rc)
        t2 = time.perf_counter()
        oc.contract(N, mN, n)
        oc.contract(R, mR, n)
        t3 = time.perf_counter()
        one = (t1 - t0) + (ns / k) * (t2 - t1) + (oc.num_tuples(ns, n) / oc.num_tuples(k, n)) * (t3 - t2)
        count = sum(1 for gg, _ in sizes if gg == g)
        parts["%d^3" % g] = round(one, 3)
        total += count * one
    return dict(value=2 * ns * len(sizes) / total, unit="shell-convs/s", cores=len(os.sched_getaffinity(0)),
                kind="oracle",
                sample=("one mock of each grid size: full mapping, convolution of both fields with %d of %d "
                        "shells, summation (n=%d) over the %d tuples of those shells; extrapolated to %d shells, "
                        "%d tuples and the batch's %d mocks" % (k, ns, n, oc.num_tuples(k, n), ns,
                                                                 oc.num_tuples(ns, n), len(sizes))),
                sample_seconds=round(time.perf_counter() - t_all, 2),
                extrapolated_step_seconds=round(total, 2), mock_seconds=parts)


def time_batch(ctx, stream, torch, steps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        e0.record(stream)
        for _ in range(steps):
            ctx.batch_launch()
        e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_mocks(args):
    """A batch of 64 independent periodic mocks (grids of 96..256 cells a side,
    50k..400k Neyman-Scott points + 10x uniform randoms each, 16 shells 10..85,
    n = 3, mixed precision), planned once and replayed as one HIP graph.  Mocks
    on one grid size run as size classes: every stage one launch for a chunk
    of mocks.  One step = the whole batch; value = shell convolutions per
    second (2 x 16 per mock).  The float64 batch (job by job) is timed beside it."""
    import torch
    import paper_2108_00015_amd as ck
    import synth
    sizes = synth.mock_sizes(64, 400)
    t = time.perf_counter()
    cats = [synth.mock_catalog(j, g, n) for j, (g, n) in enumerate(sizes)]
    npts = sum(len(d) + len(r) for d, r in cats)
    log("64 mocks: %d points in %.1f s" % (npts, time.perf_counter() - t))
    dev = torch.device("cuda:0")
    radii = synth.MOCK_RADII
    ns = len(radii)
    pos = [(torch.from_numpy(d.pos).to(dev), torch.from_numpy(r.pos).to(dev)) for d, r in cats]

    def build(dt, prec, own):
        stream = torch.cuda.Stream()
        ctx = ck.Context(0, stream=stream)
        gmax = max(g for g, _ in sizes) ** 3
        shared = (torch.empty(gmax, dtype=dt, device=dev), torch.empty(gmax, dtype=dt, device=dev))
        kspecs, jobs = {}, []
        for (g, _), (dp, rp) in zip(sizes, pos):
            grid = ck.Grid((g, g, g), (0.0, 0.0, 0.0), 5.0)
            if g not in kspecs:
                kspecs[g] = ctx.make_shell_kernels(grid, radii, dt)[0]
            kw = {} if own else dict(N=shared[0], R=shared[1])
            # no map buffers: the library keeps the maps it needs in its workspace
            jobs.append(ck.make_job(grid, kspecs[g], args.n, prec, dp, rp, fused=True, **kw))
        return ctx, stream, jobs

    ctx, stream, jobs = build(torch.float32, args.prec, True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    ctx.batch_plan(jobs)
    layout = ctx.batch_layout()
    log("plan (one eager pass, allocations): %.2f s; chunks %s" % (time.perf_counter() - t, layout))
    tuned = None
    if not args.no_autotune:
        t = time.perf_counter()
        chosen = ctx.batch_autotune(reps=2)
        tuned = {}
        for (g, _), c in zip(sizes, chosen):   # a chunk's jobs share its setting
            tuned.setdefault("%d^3" % g, c)
        log("autotune: %.2f s, %s" % (time.perf_counter() - t, tuned))
    ctx.batch_capture()
    for _ in range(args.warmup):
        ctx.batch_launch()
    ctx.synchronize()
    ms = time_batch(ctx, stream, torch, args.steps)
    log("  %.2f ms per batch of 64 mocks" % ms)
    # per-kind launch times of one eager pass (outside the timed region)
    ctx.profile(True)
    ctx.batch_run()
    ctx.synchronize()
    prof = ctx.profile_read()
    ctx.profile(False)
    chunks = {}
    for (g, _), ch in zip(sizes, layout):
        if ch >= 0:
            chunks.setdefault(ch, [g, 0])[1] += 1
    npj = [len(d) + len(r) for d, r in cats]
    stages, over_peak = {}, []
    nb = ns if "fused_zinv_contract" in prof else 8   # the fused summation transforms every radius at once
    for kind, (launches, tot) in prof.items():
        ent = dict(launches=launches, ms=round(tot, 3), avg_launch_ms=tot / launches)
        b = mock_stage_bytes(kind, sizes, ns, npj, nb)
        if b is not None:
            gbs = b / (tot * 1e-3) / 1e9
            if gbs > HBM_PEAK_GBS:
                over_peak.append(kind)
            else:
                ent["gbs"] = round(gbs, 1)
                ent["bytes_per_launch"] = b / launches
        stages[kind] = ent
    roof = roofline_of(stages, args.n, "split_bf16", MOCKS_NAME, time_key="ms",
                       note="launches of one kind differ in grid size; per-launch figures are batch averages")
    xi32 = [j.xi.cpu().numpy() for j in jobs]
    wd32 = [j.W_delta.cpu().numpy() for j in jobs]
    ctx.close()
    del jobs
    torch.cuda.empty_cache()

    ms64, rel = None, None
    if not args.no_fp64:
        log("float64 batch (job by job, shared grids, one HIP graph)")
        ctx64, stream64, jobs64 = build(torch.float64, "f64", False)
        ctx64.batch_plan(jobs64)
        ctx64.batch_capture()
        ctx64.batch_launch()
        ctx64.synchronize()
        ms64 = time_batch(ctx64, stream64, torch, max(1, min(args.steps, 3)))
        log("  %.2f ms per float64 batch" % ms64)
        wd64 = [j.W_delta.cpu().numpy() for j in jobs64]
        rel = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(wd32, wd64))
        ctx64.close()
        del jobs64
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, one mock per grid size, bounded sample)")
        cpu = mocks_cpu_baseline(sizes, cats, radii, args.n)
        log("  %.3f shell-convs/s on %d cores" % (cpu["value"], cpu["cores"]))

    total_cells = sum(g ** 3 for g, _ in sizes)
    n_alone = sum(1 for ch in layout if ch < 0)
    line = {
        "metric": "shell-convs/s over a batch of 64 mocks (graph replay)",
        "value": round(2 * ns * len(sizes) / (ms / 1e3), 3),
        "unit": "shell-convs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": MOCKS_NAME, "n_mocks": len(sizes), "grids": sorted({g for g, _ in sizes}),
                   "total_cells": total_cells, "points": npts, "n_radii": ns, "n": args.n,
                   "summation": args.prec, "fft": "f32",
                   "execution": "size classes (%d chunks: %s), %d mocks alone; one HIP graph per batch" % (
                       len(chunks), ", ".join("%d x %d^3" % (m, g) for g, m in chunks.values()), n_alone),
                   "launch_settings": tuned if tuned else "defaults"},
        "fp64_ms_per_step": round(ms64, 3) if ms64 else None,
        "fp64_over_mixed": round(ms64 / ms, 3) if ms64 else None,
        "mixed_vs_fp64_rel_W_delta": rel,
        "roofline": roof, "cpu_baseline": cpu, "stages_eager": stages, "stages_over_peak": over_peak,
        "launches_per_batch": int(sum(v["launches"] for v in stages.values())),
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cap512_ns800k_r30")
    ap.add_argument("--n", type=int, default=3)
    ap.add_argument("--prec", default="split_bf16", choices=["split_bf16", "f32", "split_f16"])
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--mode", default="npcf", choices=["npcf", "diag", "pair2"],
                    help="npcf: all tuples of order n; diag: equidistant sums for orders 2..n without maps; "
                         "pair2: n = 2 from the spectra")
    ap.add_argument("--no-autotune", action="store_true",
                    help="mock batches: keep the default launch settings instead of timing them per grid shape")
    ap.add_argument("--field-at-a-time", action="store_true",
                    help="separate path with one maps buffer, N then R (large grids)")
    ap.add_argument("--tune", default="",
                    help="launch settings for the single-catalog workloads, e.g. x_resident=3,radius_batch=15 "
                         "(conker_tune fields; default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the hot path is measured on a single MI355X "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == MOCKS_NAME:
        bench_mocks(args)
        return

    import torch
    import paper_2108_00015_amd as ck
    import synth

    w = synth.workload(args.workload)
    t = time.perf_counter()
    data, rand = w.make()
    log("catalogs: %d data + %d randoms in %.1f s" % (len(data), len(rand), time.perf_counter() - t))
    dev = torch.device("cuda:0")
    dpos = torch.from_numpy(data.pos).to(dev)
    rpos = torch.from_numpy(rand.pos).to(dev)
    dw = torch.from_numpy(data.w).to(dev) if data.w is not None else None
    rw = torch.from_numpy(rand.w).to(dev) if rand.w is not None else None
    grid = ck.Grid(w.dims, w.origin, w.cell)
    ctx = ck.Context(0)
    if args.tune:
        ctx.set_tune(**{k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))})
    ns = len(w.radii)
    nc = grid.n_cells
    kel = ck.kspec_elems(grid)

    log("mixed path (float32 FFT, %s summation): warmup %d, steps %d" % (args.prec, args.warmup, args.steps))
    mixed = run_path(ck, torch, ctx, grid, w, dpos, dw, rpos, rw, args.n, torch.float32, args.prec,
                     args.steps, args.warmup, True, args.mode, args.field_at_a_time)
    log("  %.2f ms/step" % mixed["ms"])
    fp64 = None
    if not args.no_fp64:
        log("float64 path: warmup %d, steps %d" % (args.warmup, args.steps))
        fp64 = run_path(ck, torch, ctx, grid, w, dpos, dw, rpos, rw, args.n, torch.float64, "f64",
                        args.steps, args.warmup, True, args.mode, args.field_at_a_time)
        log("  %.2f ms/step" % fp64["ms"])

    batch = min(int(os.environ.get("CONKER_RADIUS_BATCH", str(ns))), ns)
    order = mixed["axis_order"]
    fx, fl, fb = support_fractions(w, data, rand, order)
    if args.field_at_a_time:   # conker_convolve_shells: every slab and line, full maps
        fx = fl = 1.0
    pruned_fwd = args.mode != "pair2" and not args.field_at_a_time
    stages = {}
    over_peak = []
    for kind, (launches, tot) in mixed["prof"].items():
        per_step = tot / args.steps
        b = kernel_bytes(kind, launches, nc, ns, kel, len(data), len(rand), data.w is not None, 4, batch, fx, fl,
                         pruned_fwd)
        if kind == "support" and "axis_order" in mixed["prof"]:
            # built from the axis-order projections: line mask, slab counts and list written
            b = (launches / args.steps) * (nc ** (2.0 / 3.0)) * 5
        if kind == "contract_mm":   # maps and field of both fields, on the summed blocks
            b = 2 * (ns + 1) * fb * nc * 4
        ent = dict(launches_per_step=launches / args.steps, ms_per_step=per_step,
                   avg_launch_ms=tot / launches)
        if b is not None:
            gbs = b / (per_step * 1e-3) / 1e9
            if gbs > HBM_PEAK_GBS:   # the byte model overstates this kernel's traffic: no figure
                over_peak.append(kind)
                log("  stage %s: %.0f GB/s from the byte model exceeds the HBM peak; not reported" % (kind, gbs))
            else:
                ent["gbs"] = gbs
                ent["bytes_per_launch"] = b / (launches / args.steps)
        stages[kind] = ent
    # matrix-core use of the separate summation (orders n >= 3)
    if "contract_mm" in stages and args.n >= 3:
        tiles = summation_tiles(ns, args.n)
        issued = 2.0 * tiles * 1024 * fb * nc * TERM_PRODUCTS[args.prec]       # per field, summed blocks
        per_launch_ms = stages["contract_mm"]["avg_launch_ms"]
        tflops = issued / (per_launch_ms * 1e-3) / 1e12
        ent = stages["contract_mm"]
        ent["mfma_tiles"] = tiles
        ent["mfma_issued_tflops"] = round(tflops, 2)
        ent["mfma_frac_of_peak"] = round(tflops / MFMA_PEAK_TFLOPS[args.prec], 4)
        ent["tuple_cells_per_s"] = round(comb_tuples(ns, args.n) * fb * nc / (per_launch_ms * 1e-3), 1)
    # dominant kernel: largest time per step
    roof = roofline_of(stages, args.n, args.prec, w.name)

    cpu = None
    if not args.no_cpu:
        log("cpu baseline (oracle, bounded sample)")
        cpu = cpu_baseline(w, data, rand, args.n, sample_radii=4)
        log("  %.3f shell-convs/s on %d cores" % (cpu["value"], cpu["cores"]))

    s_mixed = mixed["ms"] / 1e3
    line = {
        "metric": METRIC,
        "value": round(2 * ns / s_mixed, 3),
        "unit": "shell-convs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": list(w.dims), "cell": w.cell, "n_radii": ns,
                   "radii": [w.radii[0], w.radii[-1]], "n": args.n, "n_data": len(data),
                   "n_randoms": len(rand), "weights": "log-normal sigma 0.2" if data.w is not None else "unit",
                   "summation": args.prec, "fft": "f32", "mode": args.mode,
                   "maps": ("never stored" if (args.mode != "npcf" or stages_use_fused(mixed["prof"]))
                            else ("one field at a time" if args.field_at_a_time
                                  else "carrying lines, in the workspace")),
                   "axis_order": "".join("xyz"[a] for a in AXIS_ORDERS[order]),
                   "carrying_lines": round(fl, 4), "first_axis_slabs": round(fx, 4),
                   "summed_blocks": round(fb, 4),
                   **({"tune": args.tune} if args.tune else {})},
        "s_to_W3_mixed": round(s_mixed, 5),
        "s_to_W3_fp64": round(fp64["ms"] / 1e3, 5) if fp64 else None,
        "fp64_over_mixed": round(fp64["ms"] / mixed["ms"], 3) if fp64 else None,
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_mixed": stages,
        "stages_over_peak": over_peak,
    }
    if fp64:
        st64 = {}
        for kind, (launches, tot) in fp64["prof"].items():
            st64[kind] = dict(launches_per_step=launches / args.steps, ms_per_step=tot / args.steps)
        line["stages_fp64"] = st64
        # agreement of the two GPU paths on this workload (relative to the largest entry)
        line["mixed_vs_fp64_rel"] = {
            "W_delta": float(np.abs(mixed["Wd"] - fp64["Wd"]).max() / np.abs(fp64["Wd"]).max()),
            "W_rand": float(np.abs(mixed["Wr"] - fp64["Wr"]).max() / np.abs(fp64["Wr"]).max()),
        }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
