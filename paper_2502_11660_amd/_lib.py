"""ctypes view of libmsm_gfx950.so (the C ABI in include/msm.h).

This module only loads the library and declares argument types.  There is no
fallback: if the library is missing or fails to load, every call raises.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MSM_LIB_PATH selects another build of the same library (e.g. a variant
# compiled with different kernel options); default: the in-tree build.
LIB_PATH = os.environ.get("MSM_LIB_PATH") or os.path.join(HERE, "libmsm_gfx950.so")

MSM_OK = 0
MSM_EINVAL = -1
MSM_ENOSPC = -2
MSM_EHIP = -3
MSM_FLAG_RANGE = 1
MSM_FLAG_OFFCURVE = 2
MSM_FLAG_EXCEPT = 4
MSM_FORM_XYTZ = 0
MSM_FORM_XYU = 1
MSM_RESULT_WORDS = 32
MSM_MB_MAD64 = 0
MSM_MB_ADDC = 1
MSM_MB_COPY = 2
MSM_MB_MAD64_LONE = 3
MSM_MB_MAD64_DEP = 4
MSM_MB_FEMUL_DEP = 5
MSM_DIGITS_SIGNED = 0
MSM_DIGITS_UNSIGNED = 1
MSM_DIGITS_GLV = 2
MSM_UNIT_QUAD = 0
MSM_UNIT_LANE = 1
MSM_UNIT_WIDE = 2
MSM_MUL_MONT = 0
MSM_MUL_BARRETT = 1
MSM_MUL_KARATSUBA = 2
MSM_MUL_WIDE = 3
MSM_MUL_F28 = 4
MSM_NOALLOC_SCRATCH_BYTES = 128 << 20
MSM_PROFILE_OFF = 0
MSM_PROFILE_PHASES = 1
MSM_PROFILE_ACCUM_KERNEL = 2


class MsmJob(ctypes.Structure):
    """struct msm_job"""
    _fields_ = [("xyu", ctypes.c_void_p), ("scalars", ctypes.c_void_p),
                ("result", ctypes.c_void_p), ("n", ctypes.c_size_t), ("c", ctypes.c_int),
                ("chunk", ctypes.c_int), ("tree_quad", ctypes.c_int), ("tree_wide", ctypes.c_int)]

# every exported symbol and its (restype, argtypes)
_P = ctypes.c_void_p
_SZ = ctypes.c_size_t
_I = ctypes.c_int
SIGNATURES = {
    "msm_padd_batch": (_I, [_P, _P, _P, _SZ, _I, _P]),
    "msm_fe_mul_batch": (_I, [_P, _P, _P, _SZ, _I, _P]),
    "msm_points_prepare": (_I, [_P, _P, _P, _SZ, _P, _P]),
    "msm_points_prepare_endo": (_I, [_P, _P, _P, _SZ, _P, _P]),
    "msm_gen_points": (_I, [_P, _SZ, _P, _P, _P]),
    "msm_num_windows": (_I, [_I, _I]),
    "msm_workspace_bytes": (_SZ, [_SZ, _I, _I]),
    "msm_default_window": (_I, [_SZ]),
    "msm_window_bits": (_I, [_I, _I]),
    "msm_bucket_accumulate": (_I, [_P, _P, _SZ, _I, _I, _P, _P, _SZ, _P]),
    "msm_run": (_I, [_P, _P, _SZ, _I, _I, _P, _P, _SZ, _P]),
    "msm_run_noalloc": (_I, [_P, _P, _SZ, _I, _I, _P, _P]),
    "msm_batch_workspace_bytes": (_SZ, [ctypes.POINTER(MsmJob), _SZ, _I]),
    "msm_batch_create": (_I, [ctypes.POINTER(MsmJob), _SZ, _I, _P, _SZ, _I,
                              ctypes.POINTER(ctypes.c_void_p)]),
    "msm_batch_run": (_I, [_P, _P]),
    "msm_batch_destroy": (_I, [_P]),
    "msm_server_create": (_I, [_SZ, _I, _I, ctypes.POINTER(ctypes.c_void_p)]),
    "msm_server_submit": (_I, [_P, ctypes.POINTER(MsmJob), _P, ctypes.POINTER(ctypes.c_uint64)]),
    "msm_server_progress": (_I, [_P, ctypes.POINTER(ctypes.c_uint64), _SZ,
                                 ctypes.POINTER(ctypes.c_size_t)]),
    "msm_server_drain": (_I, [_P]),
    "msm_server_stats": (_I, [_P, ctypes.POINTER(ctypes.c_size_t),
                              ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    "msm_server_destroy": (_I, [_P]),
    "msm_padd_chain": (_I, [_P, _SZ, _I, _P, _P]),
    "msm_fe_mul_chain": (_I, [_P, _P, _P, _SZ, _I, _I, _P]),
    "msm_accumulate_stream": (_I, [_P, _SZ, _SZ, _P, _P]),
    "msm_last_hip_error": (_I, []),
    "msm_status_string": (ctypes.c_char_p, [_I]),
    "msm_constants": (_I, [_P, _SZ]),
    "msm_profile_enable": (_I, [_I]),
    "msm_microbench": (_I, [_I, _SZ, _P, _SZ, _P]),
    "msm_profile_read": (_I, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_int)]),
}

_lib = None


class MSMError(RuntimeError):
    def __init__(self, fn, code, lib):
        msg = lib.msm_status_string(code).decode()
        if code == MSM_EHIP:
            msg += " (hipError_t %d)" % lib.msm_last_hip_error()
        super().__init__("%s failed: %s" % (fn, msg))
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "HIP library %s is not built; run `python -c 'import __graft_entry__ as g; g.build()'`"
                % LIB_PATH)
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(fn_name, code):
    if code != MSM_OK:
        raise MSMError(fn_name, code, lib())
    return code
