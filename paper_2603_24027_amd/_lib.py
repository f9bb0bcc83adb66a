"""ctypes view of the C ABI declared in include/fdtd.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd_mi355x.so")

FDTD_OK = 0
FDTD_EINVAL = -1
FDTD_ECFL = -2
FDTD_EREGION = -3
FDTD_ESTORE = -4
FDTD_ESTATE = -5
FDTD_EHIP = -6
FDTD_ENONFINITE = -7

STORE_FP32 = 0
STORE_FP16 = 1
STORE_BF16 = 2
STORE_FP8_E4M3_SCALED = 3
STORE_FP8_E4M3B11FNUZ = 4
STORE_FP8_E5M2FNUZ = 5
STORE_FP8_E4M3FNUZ = 6
STORE_FP8_E4M3 = 7
STORE_FP8_E3M4 = 8
STORE_FP8_E4M3FN = 9

I3 = ctypes.c_int32 * 3


class FdtdProblem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("pml", ctypes.c_int32),
        ("steps", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("courant", ctypes.c_double),
        ("pml_order", ctypes.c_int32),
        ("pml_sigma_scale", ctypes.c_double),
        ("pml_kappa_max", ctypes.c_double),
        ("pml_alpha_max", ctypes.c_double),
        ("src_comp", ctypes.c_int32),
        ("src_lo", I3), ("src_hi", I3),
        ("src_wave", ctypes.POINTER(ctypes.c_float)),
        ("src_profile", ctypes.POINTER(ctypes.c_float)),
        ("det_lo", I3), ("det_hi", I3),
        ("des_lo", I3), ("des_hi", I3),
        ("loss", ctypes.c_int32),
        ("msrc_comp", ctypes.c_int32),
        ("msrc_lo", I3), ("msrc_hi", I3),
        ("msrc_wave", ctypes.POINTER(ctypes.c_float)),
        ("msrc_profile", ctypes.POINTER(ctypes.c_float)),
    ]


class FdtdStoreCfg(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("k", ctypes.c_int32), ("interp", ctypes.c_int32)]


INTERP_LINEAR = 1
INTERP_CUBIC = 3


class FdtdStoreInfo(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "cells", "slices", "values_per_slice", "payload_bytes", "scale_bytes", "store_bytes",
        "fields_bytes", "psi_bytes", "adj_psi_bytes", "workspace_bytes", "design_cells")]


class FdtdRecord(ctypes.Structure):
    _fields_ = [("problem_hash", ctypes.c_uint64), ("dtype", ctypes.c_int32), ("k", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("consumed", ctypes.c_int32)]


class FdtdKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double)]


EXPORTS = ("store_config", "fdtd_forward", "fdtd_forward_noalloc", "fdtd_backward", "fdtd_codec_roundtrip",
           "fdtd_timing_enable", "fdtd_timing_read", "fdtd_set_graphs", "fdtd_strerror", "fdtd_last_error")
NOALLOC_SCRATCH_BYTES = 64 << 20

_lib = None


class FdtdError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__("%s (code %d): %s" % (_strerror(code), code, message))
        self.code = code


def load() -> ctypes.CDLL:
    """Load the built HIP library; there is no other implementation to fall back to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("HIP library %s is not built; run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P = ctypes.POINTER
    lib.store_config.argtypes = [P(FdtdProblem), P(FdtdStoreCfg), P(FdtdStoreInfo)]
    lib.fdtd_forward.argtypes = [P(FdtdProblem), P(FdtdStoreCfg), vp, vp, vp, vp, vp, vp, vp, P(FdtdRecord), vp]
    lib.fdtd_forward_noalloc.argtypes = [P(FdtdProblem), P(FdtdStoreCfg), vp, vp, vp, vp, vp, vp, P(FdtdRecord), vp]
    lib.fdtd_backward.argtypes = [P(FdtdProblem), P(FdtdStoreCfg), vp, vp, vp, vp, vp, vp, vp, vp,
                                  P(FdtdRecord), vp]
    lib.fdtd_codec_roundtrip.argtypes = [ctypes.c_int32, vp, ctypes.c_int64, ctypes.c_int64, vp, vp, vp, vp]
    lib.fdtd_timing_enable.argtypes = [ctypes.c_int32]
    lib.fdtd_set_graphs.argtypes = [ctypes.c_int32]
    lib.fdtd_timing_read.argtypes = [P(FdtdKernelTime), ctypes.c_int32]
    for name in ("store_config", "fdtd_forward", "fdtd_forward_noalloc", "fdtd_backward", "fdtd_codec_roundtrip",
                 "fdtd_timing_enable", "fdtd_timing_read", "fdtd_set_graphs"):
        getattr(lib, name).restype = ctypes.c_int
    lib.fdtd_strerror.argtypes = [ctypes.c_int]
    lib.fdtd_strerror.restype = ctypes.c_char_p
    lib.fdtd_last_error.argtypes = []
    lib.fdtd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _strerror(code: int) -> str:
    return load().fdtd_strerror(code).decode()


def check(code: int) -> int:
    if code < 0:
        raise FdtdError(code, load().fdtd_last_error().decode())
    return code
