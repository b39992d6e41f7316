"""ctypes declarations of the C-ABI in include/eu.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeu.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "eu.h")

EU_OK, EU_EINVAL, EU_ENOMEM, EU_EHIP, EU_ENONPHYS, EU_ESTATE = range(6)
EU_FP64, EU_FP32 = 0, 1
EU_BC_TRANSMISSIVE, EU_BC_PERIODIC = 0, 1
EU_DT_GLOBAL, EU_DT_LTS = 0, 1
EU_RESTRICT, EU_PROLONG, EU_GHOST = 0, 1, 2
EU_IC_QUADRANT, EU_IC_ELLIPSOID, EU_IC_RIEMANN1D, EU_IC_UNIFORM = 0, 1, 2, 3
EU_SCHEME_MR, EU_SCHEME_AMR = 0, 1
EU_CRIT_MR, EU_CRIT_GRADIENT = 0, 1
EU_RK_MIDPOINT, EU_RK_HEUN = 0, 1
EU_AUSM_MEAN, EU_AUSM_CRITICAL = 0, 1
EU_TILER_BLOCKS, EU_TILER_BR = 0, 1
EU_CFL_SUM, EU_CFL_MAX = 0, 1
EU_STAGE_SCHEDULES = 10
EU_STRIP_SCHEDULE0 = 6

STATUS_NAMES = {0: "EU_OK", 1: "EU_EINVAL", 2: "EU_ENOMEM", 3: "EU_EHIP", 4: "EU_ENONPHYS",
                5: "EU_ESTATE"}


class EuConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("precision", C.c_int), ("gamma", C.c_double),
        ("lo", C.c_double), ("hi", C.c_double), ("n0", C.c_int), ("levels", C.c_int),
        ("bc", C.c_int), ("cfl", C.c_double), ("t_end", C.c_double), ("eps", C.c_double),
        ("eta", C.c_double), ("patch_min", C.c_int), ("patch_max", C.c_int),
        ("time_mode", C.c_int), ("n_instances", C.c_int),
        ("inst_side_host", C.POINTER(C.c_int32)), ("stream", C.c_void_p), ("scheme", C.c_int),
        ("criterion", C.c_int), ("eps_p", C.c_double), ("eps_levels", C.c_int), ("rk", C.c_int),
        ("ausm_speed", C.c_int),
        ("tiler", C.c_int),
        ("cfl_mode", C.c_int),
        ("regrid_every", C.c_int),
    ]


class EuProblem(C.Structure):
    _fields_ = [
        ("kind", C.c_int), ("quad", (C.c_double * 4) * 4), ("x0", C.c_double), ("y0", C.c_double),
        ("ell", C.c_double * 8), ("ell_states", C.c_double * 4), ("lr", C.c_double * 6),
        ("axis", C.c_int), ("split", C.c_double), ("uniform", C.c_double * 5),
        ("inst_quad_host", C.POINTER(C.c_double)),
    ]


# name -> (restype, argtypes); every entry point declared in include/eu.h
_vp, _dp, _i64p, _u8p, _i32p, _ip = (C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                     C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.POINTER(C.c_int))
SIGNATURES = {
    "eu_query_sizes": (C.c_int, [C.POINTER(EuConfig), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "eu_create": (C.c_int, [C.POINTER(EuConfig), _vp, C.c_size_t, _vp, C.c_size_t, C.POINTER(_vp)]),
    "eu_destroy": (C.c_int, [_vp]),
    "eu_init_state": (C.c_int, [_vp, C.POINTER(EuProblem)]),
    "eu_set_finest": (C.c_int, [_vp, C.c_int, _dp]),
    "eu_mr_decompose": (C.c_int, [_vp]),
    "eu_mr_flag": (C.c_int, [_vp, C.c_double, _i64p]),
    "eu_project": (C.c_int, [_vp, C.c_int]),
    "eu_cfl_dt": (C.c_int, [_vp, C.c_double, C.c_double, _vp, _dp]),
    "eu_fv_step": (C.c_int, [_vp, _vp, C.c_int]),
    "eu_step": (C.c_int, [_vp, C.c_int]),
    "eu_advance": (C.c_int, [_vp, C.c_int, C.c_int, _ip]),
    "eu_conserved_totals": (C.c_int, [_vp, _vp, _dp]),
    "eu_conserved_totals_static": (C.c_int, [_vp, _vp]),
    "eu_copy_level": (C.c_int, [_vp, C.c_int, C.c_int, C.c_int, _dp]),
    "eu_copy_uniform": (C.c_int, [_vp, _dp]),
    "eu_get_active": (C.c_int, [_vp, C.c_int, _u8p]),
    "eu_get_flags": (C.c_int, [_vp, C.c_int, _u8p]),
    "eu_get_details": (C.c_int, [_vp, C.c_int, _dp]),
    "eu_patch_table": (C.c_int, [_vp, _i32p, C.c_int, _ip]),
    "eu_counters": (C.c_int, [_vp, _i64p, _i64p]),
    "eu_leaf_updates": (C.c_int, [_vp, _i64p, _ip]),
    "eu_time": (C.c_int, [_vp, _dp, _dp]),
    "eu_profile": (C.c_int, [_vp, C.c_int]),
    "eu_kernel_time": (C.c_int, [_vp, _dp, _i64p]),
    "eu_autotune": (C.c_int, [_vp, C.c_int, _ip, C.POINTER(C.c_float)]),
    "eu_stage_time": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_float), _i64p, _ip]),
    "eu_set_variant": (C.c_int, [_vp, C.c_int]),
    "eu_status": (C.c_int, [_vp]),
    "eu_clear_status": (C.c_int, [_vp]),
    "eu_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def load():
    """Load the in-tree libeu.so.  Raises if it has not been built: there is
    no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_1603_05211_amd.build or __graft_entry__.build())")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
