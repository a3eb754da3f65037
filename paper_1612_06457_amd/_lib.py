"""ctypes loader for libcvamx.so (argument marshalling only).

torch is imported first so that the HIP runtime the library links against
(libamdhip64.so.7) resolves to the copy torch has already loaded: one HIP
runtime per process.  There is no fallback: if the library is missing the
import of any compute entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime before libcvamx)

# CVAMX_LIB_PATH selects another build of the same library (the host-sanitizer
# build the tests make); by default the in-tree one.
LIB_PATH = os.environ.get("CVAMX_LIB_PATH") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libcvamx.so")

OK = 0
E_INVALID_ARG = -1
E_UNSUPPORTED = -2
E_EMPTY_CLASS = -3
E_NOT_PD = -4
E_DEVICE = -5
E_NO_MEMORY = -6
E_NUMERIC = -7

DT_U16, DT_F32, DT_BF16, DT_F16, DT_U8 = 0, 1, 2, 3, 4
PREC = {"fp32": 0, "bf16x3": 1, "f16x3": 2}


class CvamxError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"cvamx status {status}: {message}")
        self.status = status
        self.message = message


class Cube(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("height", ctypes.c_int64),
                ("width", ctypes.c_int64), ("bands", ctypes.c_int64),
                ("dtype", ctypes.c_int32)]


class Page(ctypes.Structure):
    _fields_ = [("bands", ctypes.c_void_p), ("pixels", ctypes.c_void_p), ("classes", ctypes.c_void_p),
                ("n_points", ctypes.c_int64), ("images", ctypes.c_void_p), ("W", ctypes.c_void_p),
                ("eigvals", ctypes.c_void_p), ("range", ctypes.c_void_p), ("status", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_f64 = ctypes.c_double

EXPORTS = {
    "cvamx_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int]),
    "cvamx_destroy": (None, [_vp]),
    "cvamx_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "cvamx_last_error": (ctypes.c_char_p, [_vp]),
    "cva_fit": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _i32, _i32, _f64, _i32,
                               _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cva_fit_points": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _vp, _i64, _i32, _i32, _f64, _i32,
                                      _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cva_fit_project": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _i32, _i32, _f64, _i32,
                                       _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cvamx_label_index": (ctypes.c_int, [_vp, _vp, _i64, _i32, _vp, _vp, _vp, _vp]),
    "cva_project": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _vp, _i32, _vp, _vp, _vp]),
    "cva_project_noalloc": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _vp, _i32, _vp, _vp, _vp]),
    "cvamx_project_float": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _vp, _i32, _vp, _vp]),
    "cvamx_stretch": (ctypes.c_int, [_vp, _vp, _i64, _i32, _i32, _f64, _vp, _i64, _i32, _vp, _vp, _vp]),
    "cvamx_compose_rgb": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "cvamx_bands_to_cube": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i64, _vp, _vp]),
    "cvamx_run_pages": (ctypes.c_int, [_vp, _i32, _i32, _i64, _i64, _i32, _i32, _i32, _f64, _i32, _f64, _i32,
                                       ctypes.POINTER(Page), _i32, _vp]),
    "cvamx_cluster_indices": (ctypes.c_int, [_vp, _vp, _i32, _i64, _i32, _vp, _vp, _i64, _i32, _f64,
                                             _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "pca_fit": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "cvamx_cva_pca": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _i32, _i32, _f64, _i32, _vp, _vp, _vp, _vp,
                                     _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp]),
    "pca_project": (ctypes.c_int, [_vp, ctypes.POINTER(Cube), _vp, _vp, _i32, _vp, _vp, _vp]),
    "cva_soft_forward": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _i32, _f64,
                                        _vp, _vp, _vp, _vp, _vp, _vp]),
    "cva_soft_backward": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _i64, _i32, _i32,
                                         _f64, _vp, _vp]),
    "cva_soft_update": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _f64, _vp]),
    "cva_solve_moments": (ctypes.c_int, [_vp, _vp, _vp, _i32, _i32, _f64, _i32, _vp, _vp, _vp]),
    "cvamx_sym_eig": (ctypes.c_int, [_i32, _vp, _vp, _vp]),
    "cvamx_sym_eig_top": (ctypes.c_int, [_i32, _vp, _i32, _vp, _vp]),
    "cvamx_set_plain_fp32": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cvamx_set_schedule": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cvamx_stream_read": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "cvamx_stream_mix": (ctypes.c_int, [_vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "cvamx_set_pca_standardize": (ctypes.c_int, [_vp, _i32]),
    "cvamx_profile_enable": (ctypes.c_int, [_vp, ctypes.c_int]),
    "cvamx_profile_report": (ctypes.c_int64, [_vp, ctypes.c_char_p, ctypes.c_int64]),
}

_LIB = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built; run paper_1612_06457_amd.build.build() "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(status: int, ctx=None):
    if status != OK:
        L = lib()
        msg = L.cvamx_last_error(ctx).decode() if ctx else L.cvamx_status_str(status).decode()
        raise CvamxError(status, msg)


_CTX = {}


def context(device: int):
    """Per-device library context (created on first use, kept for the
    process lifetime)."""
    if device not in _CTX:
        h = _vp()
        st = lib().cvamx_create(ctypes.byref(h), int(device))
        if st != OK:
            raise CvamxError(st, lib().cvamx_status_str(st).decode())
        _CTX[device] = h
    return _CTX[device]
