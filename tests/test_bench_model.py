"""Host-side pins of the bench's measurement model (CPU): the tile and tuple
counts behind the matrix-core figures, the byte model of the pruned passes,
and the choice of roofline (HBM or matrix cores) for the dominant kernel."""
import itertools
import math

import pytest

import bench


def _tiles_by_bounds(ns, n, ts=32):
    """Tiles of the order-n summation counted a second way: a tile (I, J) is
    issued iff some tuple a1 <= ... <= a_{n-1} has its row item in row block I
    and its column item in column block J, i.e. iff the smallest last radius of
    its row block is at most the largest first radius of its column block (then
    the pair of those two items, completed in between, is such a tuple).  Row
    pairs in the library's order (by their larger radius), column pairs
    lexicographic."""
    singles = [(a,) for a in range(ns)]
    pairs = [(a, b) for a in range(ns) for b in range(a, ns)]
    rows = sorted(pairs, key=lambda p: (p[1], p[0]))
    left, right = {3: (singles, singles), 4: (rows, singles), 5: (rows, pairs)}[n]
    lb = [left[i:i + ts] for i in range(0, len(left), ts)]
    rb = [right[j:j + ts] for j in range(0, len(right), ts)]
    count = 0
    for rblk in lb:
        lo = min(t[-1] for t in rblk)
        for cblk in rb:
            if lo <= max(t[0] for t in cblk):
                count += 1
    return count


@pytest.mark.parametrize("ns,n", [(10, 3), (30, 3), (40, 3), (64, 3), (8, 4), (30, 4), (6, 5), (20, 5), (25, 5)])
def test_summation_tiles_two_ways(ns, n):
    assert bench.summation_tiles(ns, n) == _tiles_by_bounds(ns, n)


def test_summation_tiles_known_counts():
    # one tile up to 32 radii at n = 3, the upper triangle of 2 x 2 blocks beyond
    assert bench.summation_tiles(30, 3) == 1
    assert bench.summation_tiles(40, 3) == 3
    assert bench.summation_tiles(64, 3) == 3
    # n = 5: rows ordered by their larger radius leave a staircase of tiles
    # (lexicographic rows would need 28 and 120)
    assert bench.summation_tiles(20, 5) == 19
    assert bench.summation_tiles(30, 5) == 64


@pytest.mark.parametrize("ns,n", [(5, 2), (10, 3), (30, 4), (20, 5), (1, 5)])
def test_comb_tuples_is_the_multiset_count(ns, n):
    assert bench.comb_tuples(ns, n) == len(list(itertools.combinations_with_replacement(range(ns), n - 1)))


def test_pruned_forward_bytes_scale_with_the_support():
    nc, ns, kel = 512 ** 3, 30, 257 ** 3
    args = dict(n_launch_units=1, nc=nc, ns=ns, kel=kel, n_data=0, n_rand=0, weighted=False, esize=4, batch=30)
    dense = {k: bench.kernel_bytes(k, **args) for k in ("fft_fwd_z", "fft_fwd_y", "fft_fwd_x")}
    fx, fl = 0.4375, 0.293
    pruned = {k: bench.kernel_bytes(k, fx=fx, fl=fl, pruned_fwd=True, **args) for k in dense}
    assert pruned["fft_fwd_z"] == pytest.approx(fl * dense["fft_fwd_z"])
    assert pruned["fft_fwd_y"] == pytest.approx((fl + fx) / 2 * dense["fft_fwd_y"])
    assert pruned["fft_fwd_x"] == pytest.approx((fx + 1) / 2 * dense["fft_fwd_x"])
    # the inverse passes: spectrum once per batch, kernel octant and output per radius
    x = bench.kernel_bytes("fft_inv_x_mul", fx=fx, fl=fl, **args)
    assert x == pytest.approx(nc * 8 + ns * (kel * 4 + fx * nc * 8))


def _stage(ms, launches=1, gb=None, tflops=None):
    e = dict(ms_per_step=ms, avg_launch_ms=ms / launches)
    if gb is not None:
        e["gbs"] = gb * launches / ms   # GB/s of the step's bytes
        e["bytes_per_launch"] = gb * 1e9
    if tflops is not None:
        e["mfma_issued_tflops"] = tflops
    return e


def test_roofline_hbm_for_the_dominant_pass():
    stages = {"fft_inv_x_mul": _stage(6.0, gb=17.2), "fft_inv_y": _stage(4.8, gb=23.5),
              "scatter": _stage(1.2, launches=2, gb=0.4)}
    r = bench.roofline_of(stages, 3, "split_bf16", "no_such_workload")
    assert r["bound"] == "hbm" and r["kernel"] == "fft_inv_x_mul" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(17.2e9 / 6.0e-3 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["traffic"] is None   # no counter summary for this workload


@pytest.mark.parametrize("n,prec", [(4, "split_f16"), (5, "split_bf16"), (5, "f32")])
def test_roofline_matrix_cores_for_orders_4_and_5(n, prec):
    stages = {"contract_mm": _stage(15.6, launches=2, gb=2.8, tflops=700.0), "fft_inv_y": _stage(1.0, gb=4.0)}
    r = bench.roofline_of(stages, n, prec, "no_such_workload")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["kernel"] == "contract_mm"
    assert r["peak"] == bench.MFMA_PEAK_TFLOPS[prec]
    assert r["frac"] == pytest.approx(700.0 / r["peak"], rel=1e-3)
    assert r["flops_per_launch"] == pytest.approx(700e12 * 7.8e-3)
    assert r["algorithmic_flops_per_launch"] * bench.TERM_PRODUCTS[prec] == pytest.approx(r["flops_per_launch"])


def test_roofline_order_3_summation_stays_on_hbm():
    stages = {"contract_mm": _stage(3.0, launches=2, gb=3.2, tflops=300.0)}
    r = bench.roofline_of(stages, 3, "split_bf16", "no_such_workload")
    assert r["bound"] == "hbm"


def test_roofline_none_without_a_byte_model():
    assert bench.roofline_of({}, 3, "split_bf16", "x") is None
    assert bench.roofline_of({"pair_spectral": _stage(2.1)}, 2, "split_bf16", "x") is None


def test_committed_traffic_summaries_name_their_sources():
    # every committed counter summary carries the hashes of the sources it was
    # taken from, and its kernel kind is one the byte model knows
    import glob
    import json
    import os
    paths = glob.glob(os.path.join(bench.ROOT, "profiles", "traffic_*.json"))
    assert paths
    for p in paths:
        with open(p) as f:
            t = json.load(f)
        assert t["sources"] and all(len(h) == 64 for h in t["sources"].values())
        assert bench.kernel_bytes(t["kind"], 1, 8, 1, 1, 0, 0, False, 4, 1) is not None
        assert t["fetch_factor"] > 0 and t["write_factor"] > 0 and math.isfinite(t["fetch_kib_per_dispatch"])
