"""ctypes declarations of the C ABI in include/nvp.h (argument marshalling only)."""

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libnvp.so")


class Medium(ctypes.Structure):
    _fields_ = [("c0", ctypes.c_double), ("rho0", ctypes.c_double), ("beta", ctypes.c_double),
                ("alpha0_db", ctypes.c_double), ("eta", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_double * 3), ("h", ctypes.c_double), ("n", ctypes.c_int64 * 3)]


class Problem(ctypes.Structure):
    _fields_ = [("med", Medium), ("f0", ctypes.c_double), ("n_harm", ctypes.c_int), ("g1", Grid),
                ("gn", ctypes.POINTER(Grid))]


# Every symbol the header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_i64p = ctypes.POINTER(ctypes.c_int64)
_st = ctypes.c_int32
_f = ctypes.c_float
_fp = ctypes.POINTER(ctypes.c_float)
SIGNATURES = {
    "nvp_status_str": (ctypes.c_char_p, [_st]),
    "nvp_last_error": (ctypes.c_char_p, [_vp]),
    "nvp_ctx_create": (_st, [_i, _vp, ctypes.POINTER(_vp)]),
    "nvp_ctx_destroy": (_st, [_vp]),
    "nvp_ctx_sync": (_st, [_vp]),
    "nvp_ctx_set_quadrature": (_st, [_vp, _i]),
    "nvp_quadrature_weights": (_st, [_i, _d, _d, _d, _dp]),
    "nvp_difference_term": (_st, [_vp, ctypes.POINTER(Grid), _vp, ctypes.POINTER(Grid), _vp, _i,
                                  ctypes.POINTER(Grid), _vp, _i, _i, _d, _i]),
    "nvp_wavenumber": (_st, [ctypes.POINTER(Medium), _d, _i, _dp, _dp]),
    "nvp_cascade_constant": (_st, [ctypes.POINTER(Medium), _d, _i, _dp]),
    "nvp_spacing": (_st, [ctypes.POINTER(Medium), _d, _i, _i, _dp]),
    "nvp_grid_from_counts": (_st, [_dp, _d, _i64p, _i64p, ctypes.POINTER(Grid)]),
    "nvp_grid_from_box": (_st, [_dp, _dp, _dp, _d, ctypes.POINTER(Grid), _i64p]),
    "nvp_rule_of_thumb_box": (_st, [_i, _d, _d, _d, _d, _dp, _dp]),
    "nvp_transfer_axis": (_st, [_d, _d, _i64, _d, _d, _i64, _i, ctypes.POINTER(ctypes.c_int32), _dp]),
    "nvp_circulant_size": (_st, [_i64, _i64p]),
    "nvp_transform_lengths": (_st, [ctypes.POINTER(ctypes.c_int32), _i, ctypes.POINTER(_i)]),
    "nvp_volume_potential": (_st, [_vp, _d, _d, ctypes.POINTER(Grid), _vp, _vp, _i]),
    "nvp_volume_potential_noalloc": (_st, [_vp, _d, _d, ctypes.POINTER(Grid), _vp, _vp, _i]),
    "nvp_volume_potential_box": (_st, [_vp, _d, _d, ctypes.POINTER(Grid), _vp, _i64p, _d, _vp, _i]),
    "nvp_field_lin3": (_st, [_vp, _i64, _vp, _vp, _vp, _vp, _dp, _dp, _i]),
    "nvp_field_diff_norms": (_st, [_vp, _i64, _vp, _vp, _i, _dp]),
    "nvp_incident_field": (_st, [_vp, _d, _d, _d, _d, _vp, ctypes.c_int64, ctypes.POINTER(Grid), _vp, _i]),
    "nvp_vie_solve": (_st, [_vp, _d, _d, ctypes.POINTER(Grid), _vp, _vp, _vp, _i, _d, _i, ctypes.POINTER(_i),
                            ctypes.POINTER(_d)]),
    "nvp_incident_at": (_st, [_vp, _d, _d, _d, _d, _vp, ctypes.c_int64, _vp, ctypes.c_int64, _vp, _i]),
    "nvp_radiated_power": (_st, [_vp, _d, _d, _d, _d, _vp, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), _d, _d, _d,
                                 _i, _i, ctypes.POINTER(ctypes.c_double)]),
    "nvp_plan_cascade": (_st, [_vp, ctypes.POINTER(Medium), _d, _i, ctypes.POINTER(Grid), ctypes.POINTER(Grid),
                               _i, _i, ctypes.POINTER(_vp)]),
    "nvp_plan_workspace_bytes": (_st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "nvp_plan_regrid": (_st, [_vp, _i, ctypes.POINTER(Grid)]),
    "nvp_plan_set_kernel_cache": (_st, [_vp, _i]),
    "nvp_plan_set_overlap": (_st, [_vp, _i]),
    "nvp_plan_work_bytes": (_st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "nvp_plan_set_workspace": (_st, [_vp, _vp, ctypes.c_size_t]),
    "nvp_execute_harmonic": (_st, [_vp, _i, ctypes.POINTER(_vp), _vp]),
    "nvp_execute_cascade": (_st, [_vp, _vp, ctypes.POINTER(_vp)]),
    "nvp_plan_destroy": (_st, [_vp]),
    "nvp_plan_set_timing": (_st, [_vp, _i]),
    "nvp_plan_get_timing": (_st, [_vp, _dp, _i64p, _i]),
    "nvp_source_term": (_st, [_vp, _i, ctypes.POINTER(_vp), _vp]),
    "nvp_plan_autotune": (_st, [_vp, ctypes.c_char_p, _i]),
    "nvp_plan_get_tuning": (_st, [_vp, _i, ctypes.POINTER(_i)]),
    "nvp_plan_set_tuning": (_st, [_vp, _i, ctypes.POINTER(_i)]),
    "nvp_batch_create": (_st, [_vp, _i, ctypes.POINTER(Problem), _i, _i, ctypes.POINTER(_vp)]),
    "nvp_batch_outputs": (_st, [_vp, _i64p]),
    "nvp_batch_set_graph": (_st, [_vp, _i, _i]),
    "nvp_batch_set_grouped": (_st, [_vp, _i]),
    "nvp_batch_autotune": (_st, [_vp, ctypes.c_char_p, _i]),
    "nvp_batch_execute": (_st, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)]),
    "nvp_batch_destroy": (_st, [_vp]),
    "nvp_qbox": (_st, [_vp, _i64p, _vp, _i, _i, _dp, _i64p]),
    "nvp_box_potential": (_st, [_vp, _d, _d, ctypes.POINTER(Grid), _vp, _i, _i64p, _i, _i64p, _dp]),
    "nvp_boxnet_create": (_st, [_vp, _i, ctypes.POINTER(_vp)]),
    "nvp_boxnet_set_params": (_st, [_vp, _fp, _i64]),
    "nvp_boxnet_get_params": (_st, [_vp, _fp, _i64]),
    "nvp_boxnet_set_norm": (_st, [_vp, _fp, _fp]),
    "nvp_boxnet_predict": (_st, [_vp, _i, _vp, _vp]),
    "nvp_boxnet_grads": (_st, [_vp, _i, _vp, _vp, _f, _vp, _fp]),
    "nvp_boxnet_train_step": (_st, [_vp, _i, _vp, _vp, _f, _f, _fp]),
    "nvp_boxnet_destroy": (_st, [_vp]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libnvp.so is not built (%s); run "
                               "python -m paper_2011_03009_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib
