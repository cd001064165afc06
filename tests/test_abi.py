"""The C-ABI library loads, exports every declared symbol, and its host-only calls
agree with the oracle.  No GPU work is issued."""
import ctypes as ct
import math
import os
import re

import pytest

from oracle import conker as oc
from paper_2108_00015_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "conker.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(conker_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for required in ("conker_grid_assign", "conker_make_shell_kernels", "conker_convolve_shells",
                     "conker_contract_npt", "conker_form_delta", "conker_ratio"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(_declared()) == set(_lib.SIGNATURES)


@pytest.mark.parametrize("ns,n", [(10, 2), (10, 3), (30, 3), (30, 4), (20, 5), (40, 3), (1, 5)])
def test_num_tuples(ns, n):
    assert _lib.load().conker_num_tuples(ns, n) == len(oc.radius_tuples(ns, n)) == math.comb(ns + n - 2, n - 1)


def test_num_tuples_rejects_order_below_two():
    assert _lib.load().conker_num_tuples(10, 1) == -1


@pytest.mark.parametrize("r", [0.5, 1.0, 2.0, 4.0, 11.0, 11.46, 20.0, 33.0])
def test_shell_size_matches_oracle(r):
    out = ct.c_int64()
    assert _lib.load().conker_shell_size(r, ct.byref(out)) == _lib.OK
    assert out.value == len(oc.shell_offsets(r))


def test_shell_size_rejects_small_radius():
    out = ct.c_int64()
    assert _lib.load().conker_shell_size(0.49, ct.byref(out)) == _lib.ERANGE


def test_kspec_elems():
    g = _lib.ConkerGrid()
    for k, v in enumerate((512, 256, 128)):
        g.dims[k] = v
    g.cell = 1.0
    assert _lib.load().conker_kspec_elems(ct.byref(g)) == 257 * 129 * 65


def test_create_without_gpu_reports_error_or_succeeds():
    """Without a GPU conker_create must fail with a status (not crash); with one it succeeds."""
    lib = _lib.load()
    h = ct.c_void_p()
    st = lib.conker_create(ct.byref(h), 0, None, 0)
    if st == _lib.OK:
        lib.conker_destroy(h)
    else:
        assert st in (_lib.EHIP, _lib.EINVAL)
        assert h.value is None
        assert len(lib.conker_last_error(None)) > 0


def test_null_context_is_rejected():
    lib = _lib.load()
    g = _lib.ConkerGrid()
    assert lib.conker_grid_assign(None, ct.byref(g), None, None, 0, _lib.F32, None, None, None) == _lib.EINVAL
    assert lib.conker_contract_npt(None, ct.byref(g), _lib.F64, None, None, 3, 3, _lib.MM_F64, None) == _lib.EINVAL
