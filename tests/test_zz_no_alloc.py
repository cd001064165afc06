"""The allocation-free equidistant summation (conker_contract_diag_noalloc),
called through the C ABI, against conker_contract_diag on the same inputs:
two calls in a row, the second on a smaller grid with fewer radii (the shared
scratch array keeps the first call's partial sums), and sizes beyond its fixed
scratch rejected."""
import ctypes as ct
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ck():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_00015_amd as m
    return m


def _inputs(dims, ns, dt, seed):
    g = torch.Generator().manual_seed(seed)
    F = torch.randn(dims, generator=g, dtype=torch.float64)
    maps = torch.randn((ns,) + tuple(dims), generator=g, dtype=torch.float64)
    return F.to(DEV, dt), maps.to(DEV, dt)


def _call(lib, ctx, fn, grid, F, maps, n_max, dt):
    ns = int(maps.shape[0])
    out = torch.full((n_max - 1, ns), np.nan, dtype=torch.float64, device=DEV)
    g = grid.c()
    st = getattr(lib, fn)(ctx.h, ct.byref(g), 2 if dt == torch.float64 else 1, ct.c_void_p(F.data_ptr()),
                          ct.c_void_p(maps.data_ptr()), ns, n_max, ct.c_void_p(out.data_ptr()))
    return st, out


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_noalloc_matches_contract_diag_two_calls(ck, dt):
    from paper_2108_00015_amd import _lib
    lib = _lib.load()
    ctx = ck.Context(0)
    cases = [((64, 64, 128), 12, 5), ((32, 32, 64), 5, 3)]   # the second call is smaller
    for dims, ns, n_max in cases:
        _say("noalloc", dt, dims, ns, n_max)
        grid = ck.Grid(dims, (0, 0, 0), 1.0)
        F, maps = _inputs(dims, ns, dt, 7 + ns)
        st0, ref = _call(lib, ctx, "conker_contract_diag", grid, F, maps, n_max, dt)
        st1, got = _call(lib, ctx, "conker_contract_diag_noalloc", grid, F, maps, n_max, dt)
        ctx.synchronize()
        assert st0 == _lib.OK and st1 == _lib.OK
        r, o = ref.cpu().numpy(), got.cpu().numpy()
        assert np.all(np.isfinite(o))
        # the same kernels over the same cut of the cells: identical sums
        assert np.array_equal(o, r), np.abs(o - r).max()
        # and the sums themselves, against float64 sums on the host
        Fh = F.double().cpu().numpy().reshape(-1)
        Mh = maps.double().cpu().numpy().reshape(ns, -1)
        if dt == torch.float32:
            tol = 1e-5
        else:
            tol = 1e-12
        for p in range(1, n_max):
            want = (Fh[None, :] * Mh ** p).sum(axis=1)
            err = np.abs(o[p - 1] - want).max() / np.abs(want).max()
            assert err <= tol, (p, err)
    ctx.close()


def test_noalloc_limit_of_its_scratch(ck):
    """256^3 float32 cells are summed by 2048 workgroups: at n_max = 5 the 4 MiB
    scratch holds the partial sums of 64 radii (accepted, identical to
    conker_contract_diag) and not of 65 (rejected before any launch)."""
    from paper_2108_00015_amd import _lib
    lib = _lib.load()
    ctx = ck.Context(0)
    dims = (256, 256, 256)
    grid = ck.Grid(dims, (0, 0, 0), 1.0)
    g = torch.Generator(device=DEV).manual_seed(11)
    F = torch.randn(dims, generator=g, device=DEV, dtype=torch.float32)
    maps = torch.randn((65,) + dims, generator=g, device=DEV, dtype=torch.float32)
    st0, ref = _call(lib, ctx, "conker_contract_diag", grid, F, maps[:64], 5, torch.float32)
    st1, got = _call(lib, ctx, "conker_contract_diag_noalloc", grid, F, maps[:64], 5, torch.float32)
    ctx.synchronize()
    assert st0 == _lib.OK and st1 == _lib.OK
    assert torch.equal(ref, got)
    st, _ = _call(lib, ctx, "conker_contract_diag_noalloc", grid, F, maps, 5, torch.float32)
    assert st == _lib.ERANGE
    assert "allocation-free" in lib.conker_last_error(ctx.h).decode()
    del maps
    ctx.close()
    torch.cuda.empty_cache()
