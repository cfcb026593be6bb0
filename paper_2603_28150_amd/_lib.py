"""ctypes binding of libpat.so (include/pat.h).  Marshalling only.

The library is loaded from this package directory.  If it is missing or does
not load, every call raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpat.so")


class OpInfo(C.Structure):
    """pat_op_info."""
    _fields_ = [("nk", C.c_int32), ("nclass", C.c_int32), ("members_max", C.c_int32),
                ("nz_sim", C.c_int32), ("slab_bytes_A", C.c_size_t), ("slab_bytes_AT", C.c_size_t),
                ("spec_rows", C.c_int32), ("nitems", C.c_int32),
                ("read_bytes_A", C.c_size_t), ("read_bytes_AT", C.c_size_t),
                ("gram_bytes", C.c_size_t)]


class Geometry(C.Structure):
    """pat_geometry."""
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nt", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("dt", C.c_double), ("c", C.c_double),
                ("nz_sim", C.c_int32), ("h_dtype", C.c_int32), ("boundary", C.c_int32),
                ("n_ir", C.c_int32), ("ir", C.POINTER(C.c_double)),
                ("sx", C.c_int32), ("sy", C.c_int32), ("build", C.c_int32)]


H_F32, H_BF16, H_F16 = 0, 1, 2
HDTYPES = {"f32": H_F32, "bf16": H_BF16, "f16": H_F16}
BOUNDARIES = {"periodic": 0, "linear": 1}
BUILDS = {"closed": 0, "step": 1}

STATUS = {0: "PAT_OK", -1: "PAT_EINVAL", -2: "PAT_EUNSUPPORTED", -3: "PAT_ENOMEM",
          -4: "PAT_EHIP", -5: "PAT_ENONFINITE"}


class PatError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_vp, _sz, _i32, _f32, _f64 = C.c_void_p, C.c_size_t, C.c_int32, C.c_float, C.c_double
_pp = C.POINTER(C.c_void_p)

# name -> argument types (every function returns pat_status unless listed in _RESTYPES)
SIGNATURES = {
    "pat_ctx_create": [C.c_int, _pp],
    "pat_ctx_destroy": [_vp],
    "pat_H_bytes": [C.POINTER(Geometry), C.POINTER(_sz), C.POINTER(_sz)],
    "pat_H_build": [_vp, C.POINTER(Geometry), _vp, _sz, _vp, _sz, _vp, _pp],
    "pat_op_destroy": [_vp],
    "pat_H_export": [_vp, _i32, _i32, _vp, _vp],
    "pat_workspace_bytes": [_vp, _i32, C.POINTER(_sz)],
    "pat_get_info": [_vp, C.POINTER(OpInfo)],
    "pat_spectrum_rows": [_vp, C.POINTER(_i32)],
    "pat_spectrum_stride": [_i32, C.POINTER(_i32)],
    "pat_apply_A": [_vp, _vp, _vp, _i32, _vp, _sz, _vp],
    "pat_apply_AT": [_vp, _vp, _vp, _i32, _vp, _sz, _vp],
    "pat_apply_A_noalloc": [_vp, _vp, _vp, _i32, _vp],
    "pat_power_norm": [_vp, _vp, _i32, C.POINTER(_f64), C.POINTER(_f64), _vp, _sz, _vp],
    "pat_recon_fista": [_vp, _vp, _vp, _i32, _f32, _f32, _i32, _i32, _vp, _vp, _sz, _vp],
    "pat_fista_step": [_vp, _i32, _vp, _vp, _vp, C.POINTER(_f64), C.POINTER(_f32),
                       C.POINTER(_f32), C.POINTER(_i32), _vp, _vp, _sz, _vp],
    "pat_fista_step_normal": [_vp, _i32, _vp, _vp, _vp, C.POINTER(_f64), C.POINTER(_f32),
                              C.POINTER(_f32), C.POINTER(_i32), _vp, _vp, _sz, _vp],
    "pat_adjoint_check": [_vp, _vp, _vp, C.POINTER(_f64), _vp, _sz, _vp],
    "pat_spectrum": [_vp, _vp, _vp, _i32, _vp, _sz, _vp],
    "pat_inverse_spectrum": [_vp, _vp, _vp, _i32, _vp, _vp, _sz, _vp],
    "pat_contract": [_vp, _i32, _vp, _vp, _i32, _vp],
    "pat_status_str": [C.c_int],
    "pat_last_error": [],
}
_RESTYPES = {"pat_ctx_destroy": None, "pat_status_str": C.c_char_p, "pat_last_error": C.c_char_p}

_lib = None


def load(path: str = LIB_PATH):
    """Opens libpat.so once and declares every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2603_28150_amd.build`")
    lib = C.CDLL(path)
    for name, argtypes in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = _RESTYPES.get(name, C.c_int)
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        raise PatError(status, load().pat_last_error().decode())


def call(name: str, *args) -> None:
    check(getattr(load(), name)(*args))
