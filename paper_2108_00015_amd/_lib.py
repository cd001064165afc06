"""ctypes declarations of the C ABI in include/conker.h.

The shared library is built in-tree (paper_2108_00015_amd/libconker.so).  If it
is missing, loading raises: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libconker.so")

OK, EINVAL, ENOMEM, EUNSUPPORTED, EHIP, ERANGE = 0, -1, -2, -3, -4, -5
F32, F64 = 1, 2
MM_F64, MM_F32, MM_SPLIT_BF16, MM_SPLIT_F16 = 0, 1, 2, 3

STATUS_NAMES = {OK: "CONKER_OK", EINVAL: "CONKER_EINVAL", ENOMEM: "CONKER_ENOMEM",
                EUNSUPPORTED: "CONKER_EUNSUPPORTED", EHIP: "CONKER_EHIP", ERANGE: "CONKER_ERANGE"}

# name -> (restype, argtypes)
SIGNATURES = {
    "conker_create": (ct.c_int, [ct.POINTER(ct.c_void_p), ct.c_int, ct.c_void_p, ct.c_size_t]),
    "conker_destroy": (None, [ct.c_void_p]),
    "conker_set_stream": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "conker_last_error": (ct.c_char_p, [ct.c_void_p]),
    "conker_workspace_bytes": (ct.c_size_t, [ct.c_void_p]),
    "conker_grid_assign": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64,
                                      ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "conker_form_delta": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                     ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "conker_shell_size": (ct.c_int, [ct.c_double, ct.POINTER(ct.c_int64)]),
    "conker_kspec_elems": (ct.c_int64, [ct.c_void_p]),
    "conker_make_shell_kernels": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_double), ct.c_int,
                                             ct.c_int, ct.c_void_p, ct.POINTER(ct.c_int64)]),
    "conker_convolve_shells": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                          ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p]),
    "conker_num_tuples": (ct.c_int64, [ct.c_int, ct.c_int]),
    "conker_contract_npt": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                       ct.c_int, ct.c_int, ct.c_int, ct.c_void_p]),
    "conker_convolve_contract": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                            ct.c_void_p, ct.c_int, ct.c_int, ct.c_int, ct.c_void_p,
                                            ct.c_void_p]),
    "conker_contract_diag": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                        ct.c_int, ct.c_int, ct.c_void_p]),
    "conker_contract_diag_noalloc": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                                ct.c_int, ct.c_int, ct.c_void_p]),
    "conker_convolve_diag": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]),
    "conker_convolve_contract_cross": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int,
                                                  ct.c_int, ct.c_void_p, ct.c_void_p]),
    "conker_convolve_diag_cross": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                              ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_int,
                                              ct.c_void_p, ct.c_void_p]),
    "conker_ratio_cross": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                      ct.c_int64, ct.c_void_p]),
    "conker_pair_spectral": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p,
                                        ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "conker_delta_field": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                      ct.c_void_p]),
    "conker_ratio_combined": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                         ct.c_int64, ct.c_void_p, ct.c_void_p, ct.c_void_p]),
    "conker_map_ratio": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p]),
    "conker_value_histogram": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_int64, ct.c_double, ct.c_double,
                                          ct.c_int, ct.c_void_p]),
    "conker_sky_to_cartesian": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                           ct.c_int64, ct.c_void_p]),
    "conker_analytic_randoms": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int, ct.c_void_p, ct.c_double,
                                           ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                                           ct.c_int, ct.c_void_p, ct.c_void_p]),
    "conker_ratio": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int,
                                ct.c_int64, ct.c_void_p]),
    "conker_synchronize": (ct.c_int, [ct.c_void_p]),
    "conker_batch_plan": (ct.c_int, [ct.c_void_p, ct.c_void_p, ct.c_int]),
    "conker_batch_run": (ct.c_int, [ct.c_void_p]),
    "conker_batch_capture": (ct.c_int, [ct.c_void_p]),
    "conker_batch_launch": (ct.c_int, [ct.c_void_p]),
    "conker_batch_classes": (ct.c_int, [ct.c_void_p, ct.c_int]),
    "conker_batch_layout": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "conker_set_tune": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "conker_get_tune": (ct.c_int, [ct.c_void_p, ct.c_void_p]),
    "conker_batch_autotune": (ct.c_int, [ct.c_void_p, ct.c_int, ct.c_void_p]),
    "conker_axis_order_used": (ct.c_int, [ct.c_void_p, ct.POINTER(ct.c_int)]),
    "conker_profile_enable": (ct.c_int, [ct.c_void_p, ct.c_int]),
    "conker_profile_read": (ct.c_int, [ct.c_void_p, ct.c_int, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_double)]),
    "conker_profile_kind_name": (ct.c_char_p, [ct.c_int]),
}


class ConkerGrid(ct.Structure):
    _fields_ = [("dims", ct.c_int32 * 3), ("origin", ct.c_double * 3), ("cell", ct.c_double)]


class ConkerCosmology(ct.Structure):
    _fields_ = [("omega_m", ct.c_double), ("omega_k", ct.c_double), ("omega_lambda", ct.c_double),
                ("h0", ct.c_double), ("c", ct.c_double), ("z_max", ct.c_double)]


class ConkerTune(ct.Structure):
    _fields_ = [("x_tile", ct.c_int32), ("y_tile", ct.c_int32), ("x_resident", ct.c_int32),
                ("mm_kernel", ct.c_int32), ("radius_batch", ct.c_int32), ("axis_order", ct.c_int32),
                ("radix", ct.c_int32), ("ms", ct.c_float)]


class ConkerJob(ct.Structure):
    _fields_ = [("grid", ConkerGrid), ("dtype", ct.c_int), ("prec", ct.c_int), ("n", ct.c_int),
                ("n_radii", ct.c_int), ("d_kspec", ct.c_void_p),
                ("d_data_pos", ct.c_void_p), ("d_data_w", ct.c_void_p), ("n_data", ct.c_int64),
                ("d_rand_pos", ct.c_void_p), ("d_rand_w", ct.c_void_p), ("n_rand", ct.c_int64),
                ("d_N", ct.c_void_p), ("d_R", ct.c_void_p), ("d_maps_N", ct.c_void_p), ("d_maps_R", ct.c_void_p),
                ("d_wsum", ct.c_void_p), ("d_n_outside", ct.c_void_p), ("d_alpha", ct.c_void_p),
                ("d_W_delta", ct.c_void_p), ("d_W_rand", ct.c_void_p), ("d_xi", ct.c_void_p)]


_LIB = None


def load() -> ct.CDLL:
    """Loads libconker.so once; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libconker.so is not built (run: python -m paper_2108_00015_amd.build)")
        lib = ct.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB
