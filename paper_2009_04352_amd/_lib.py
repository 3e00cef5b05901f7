"""ctypes declarations of the C ABI in include/lbmwf.h (argument marshalling only).

The library is paper_2009_04352_amd/liblbmwf.so, built by
paper_2009_04352_amd/csrc/build.py.  There is no fallback: without the
built library every call raises.
"""
import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblbmwf.so")

LBM_OK = 0
LBM_E_ARG, LBM_E_STATE, LBM_E_OOM, LBM_E_DEVICE, LBM_E_NONFINITE, LBM_E_NEWTON = -1, -2, -3, -4, -5, -6
LBM_BB, LBM_WFB, LBM_FREESLIP = 0, 1, 2
LBM_STORE_F64, LBM_STORE_F32, LBM_STORE_F16, LBM_STORE_BF16 = 0, 1, 2, 3
(LBM_P_Y1, LBM_P_NEWTON_TOL, LBM_P_NEWTON_MAXIT, LBM_P_STATS_EVERY, LBM_P_STORE, LBM_P_TILE_ODD,
 LBM_P_TILE_EVEN, LBM_P_XCD_REMAP, LBM_P_GRAPH_STEPS, LBM_P_BC, LBM_P_TAU0, LBM_P_FX, LBM_P_CS,
 LBM_P_VECTOR, LBM_P_BRICK, LBM_P_ODD_ROWS, LBM_P_SPREAD, LBM_P_ODD_BY_ROWS, LBM_P_COLLISION,
 LBM_P_MRT_S_E, LBM_P_MRT_S_EPS, LBM_P_MRT_S_Q, LBM_P_MRT_S_PI, LBM_P_MRT_S_M, LBM_P_VD_APLUS,
 LBM_P_VD_UTAU, LBM_P_WALL_NODES, LBM_P_XCD_CHUNK) = range(28)
LBM_BGK, LBM_MRT = 0, 1

# every symbol the header declares, with (restype, argtypes)
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_vp = C.c_void_p


class Grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32)]


SIGNATURES = {
    "lbm_create": (C.c_int, [C.POINTER(Grid), C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                             C.POINTER(_vp)]),
    "lbm_destroy": (None, [_vp]),
    "lbm_set_param": (C.c_int, [_vp, C.c_int, C.c_double]),
    "lbm_get_param": (C.c_int, [_vp, C.c_int, _dp]),
    "lbm_required_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "lbm_bind_storage": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lbm_set_stream": (C.c_int, [_vp, _vp]),
    "lbm_set_boundary": (C.c_int, [_vp, C.c_int]),
    "lbm_init_spalding": (C.c_int, [_vp, C.c_double, C.c_double, C.c_uint64]),
    "lbm_set_state": (C.c_int, [_vp, _dp, C.c_int64]),
    "lbm_get_state": (C.c_int, [_vp, _dp]),
    "lbm_get_state_cells": (C.c_int, [_vp, C.c_int64, _i64p, _dp]),
    "lbm_step": (C.c_int, [_vp, C.c_int64]),
    "lbm_sync": (C.c_int, [_vp, _i64p]),
    "lbm_steps_done": (C.c_int, [_vp, _i64p]),
    "lbm_moments": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lbm_moments_cells": (C.c_int, [_vp, C.c_int64, _i64p, _dp]),
    "lbm_moments_device": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "lbm_wall_shear": (C.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "lbm_wall_yplus_pdf": (C.c_int, [_vp, C.c_int32, C.c_double, C.c_double, C.c_void_p, _dp]),
    "lbm_wall_yplus_pdf_noalloc": (C.c_int, [_vp, C.c_int32, C.c_double, C.c_double, C.c_void_p, C.c_void_p]),
    "lbm_init_moments": (C.c_int, [_vp, _dp, _dp]),
    "lbm_wall_mass_change": (C.c_int, [_vp, _dp, _dp]),
    "lbm_get_wall_nodes": (C.c_int, [_vp, _dp, _dp]),
    "lbm_stats_reset": (C.c_int, [_vp]),
    "lbm_stats_sums": (C.c_int, [_vp, _dp, _i64p]),
    "lbm_stats_get": (C.c_int, [_vp, _dp, _i64p]),
    "lbm_autotune": (C.c_int, [_vp, C.c_int, _i32p]),
    "lbm_spalding_uplus": (C.c_int, [C.c_double, C.c_double, C.c_double, _dp]),
    "lbm_device_wall_utau": (C.c_int, [C.c_int32, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.c_int32, _dp, _i32p]),
    "lbm_codec_roundtrip": (C.c_int, [C.c_int, C.c_int64, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "lbm_copy_probe": (C.c_int, [_vp, _vp, C.c_size_t, _vp]),
    "lbm_batch_create": (C.c_int, [C.c_int32, C.POINTER(Grid), _dp, _dp, _dp, _i32p, C.c_double, C.c_double,
                                   C.POINTER(_vp)]),
    "lbm_batch_destroy": (None, [_vp]),
    "lbm_batch_set_param": (C.c_int, [_vp, C.c_int, C.c_double]),
    "lbm_batch_required_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "lbm_batch_bind_storage": (C.c_int, [_vp, _vp, C.c_size_t]),
    "lbm_batch_set_stream": (C.c_int, [_vp, _vp]),
    "lbm_batch_init_spalding": (C.c_int, [_vp, _dp, C.c_double, C.POINTER(C.c_uint64)]),
    "lbm_batch_step": (C.c_int, [_vp, C.c_int64]),
    "lbm_batch_sync": (C.c_int, [_vp, _i64p, _i32p]),
    "lbm_batch_instance": (_vp, [_vp, C.c_int32]),
    "lbm_batch_autotune": (C.c_int, [_vp, C.c_int, _i32p]),
    "lbm_batch_last_error": (C.c_char_p, [_vp]),
    "lbm_status_str": (C.c_char_p, [C.c_int]),
    "lbm_last_error": (C.c_char_p, [_vp]),
}

_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbmwf.so is not built (run __graft_entry__.build() or "
                               "paper_2009_04352_amd/csrc/build.py): there is no fallback path")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (lib().lbm_status_str(code).decode(), code, msg))
        self.code = code


def check(code, ctx=None):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_last_error(ctx).decode())
    return code


def check_batch(code, batch=None):
    if code != LBM_OK:
        raise LbmError(code, lib().lbm_batch_last_error(batch).decode())
    return code


def dptr(a):
    """double* of a C-contiguous float64 numpy array (None -> NULL)."""
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def i64ptr(a):
    return a.ctypes.data_as(_i64p)
