"""ctypes binding of libdgswe.so (argument marshalling only).

Every function of include/dgswe.h is exposed under the same name.  The
library is loaded from this package directory; there is no fallback: if it
is missing or fails to load, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DGSWE_LIB") or os.path.join(_HERE, "libdgswe.so")

DGSWE_OK, DGSWE_EINVAL, DGSWE_ENOMEM, DGSWE_EHIP, DGSWE_ESTATE, DGSWE_ENONFINITE, DGSWE_EBUDGET = 0, -1, -2, -3, -4, -5, -6
FP64, FP32 = 0, 1
ROE, LLF = 0, 1
MANNING, QUADRATIC = 0, 1
LAND, OCEAN, RIVER, OUTFLOW = 0, 1, 2, 3
MODAL, VERTEX = 0, 1
MAX_SLOTS = 16
TUNE_STAGE_VARIANT = 1
TUNE_FUSED_POST = 2
TUNE_STAGE_TILE = 3

ERRORS = {
    DGSWE_EINVAL: "EINVAL", DGSWE_ENOMEM: "ENOMEM", DGSWE_EHIP: "EHIP",
    DGSWE_ESTATE: "ESTATE", DGSWE_ENONFINITE: "ENONFINITE", DGSWE_EBUDGET: "EBUDGET",
}


class Params(C.Structure):
    _fields_ = [("p", C.c_int32), ("precision", C.c_int32), ("flux", C.c_int32),
                ("rk_stages", C.c_int32), ("limiter", C.c_int32), ("friction", C.c_int32),
                ("cfl", C.c_double), ("dt_fixed", C.c_double), ("dt_max", C.c_double),
                ("H0", C.c_double), ("g", C.c_double)]


class Mass(C.Structure):
    _fields_ = [("t", C.c_double), ("dt_last", C.c_double), ("dt_next", C.c_double),
                ("volume", C.c_double), ("rain_in", C.c_double), ("bnd_in", C.c_double),
                ("bnd_out", C.c_double), ("steps", C.c_int64), ("n_dry", C.c_int64),
                ("n_negative", C.c_int64), ("bad_element", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DgsweError(RuntimeError):
    def __init__(self, code, func, msg):
        super().__init__(f"{func}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_F = C.POINTER(C.c_float)
_I = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_U8 = C.POINTER(C.c_uint8)

SIGNATURES = {
    "dgswe_default_params": (C.c_int, [C.POINTER(Params)]),
    "dgswe_create": (C.c_int, [C.POINTER(Params), _P, C.POINTER(_P)]),
    "dgswe_destroy": (C.c_int, [_P]),
    "dgswe_workspace_bind": (C.c_int, [_P, _P, C.c_size_t]),
    "dgswe_upload_mesh": (C.c_int, [_P, C.c_int64, _D, _D, _D, C.c_int64, _I, C.c_int64, _I, _I, _I]),
    "dgswe_share_mesh": (C.c_int, [_P, _P]),
    "dgswe_set_initial_nodal": (C.c_int, [_P, _D, _D, _D]),
    "dgswe_set_state": (C.c_int, [_P, C.c_int, _D, C.c_double, C.POINTER(Mass)]),
    "dgswe_set_rain_nodal": (C.c_int, [_P, _D]),
    "dgswe_set_rain_parametric": (C.c_int, [_P, C.c_int32, _D]),
    "dgswe_set_rain_gridded": (C.c_int, [_P, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32,
                                          C.c_int32, C.c_int32, _D, _F]),
    "dgswe_clear_rain": (C.c_int, [_P]),
    "dgswe_set_wind_vortex": (C.c_int, [_P, C.c_int32, _D]),
    "dgswe_clear_wind": (C.c_int, [_P]),
    "dgswe_set_ocean_tide": (C.c_int, [_P, C.c_int32, C.c_double, C.c_int32, _D]),
    "dgswe_set_river_flux": (C.c_int, [_P, C.c_int32, C.c_int32, _D, _D]),
    "dgswe_step": (C.c_int, [_P, C.c_int64]),
    "dgswe_step_noalloc": (C.c_int, [_P, C.c_int64]),
    "dgswe_sync": (C.c_int, [_P]),
    "dgswe_read_state": (C.c_int, [_P, C.c_int, _D]),
    "dgswe_read_flags": (C.c_int, [_P, _U8]),
    "dgswe_mass_totals": (C.c_int, [_P, C.POINTER(Mass)]),
    "dgswe_info": (C.c_int, [_P, _I64, _I64, _I64, _I64]),
    "dgswe_footprint_bytes": (C.c_int64, [C.POINTER(Params), C.c_int64, C.c_int64]),
    "dgswe_set_tuning": (C.c_int, [_P, C.c_int, C.c_int]),
    "dgswe_get_tuning": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int)]),
    "dgswe_autotune": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    "dgswe_set_profiling": (C.c_int, [_P, C.c_int]),
    "dgswe_kernel_stats": (C.c_int, [_P, C.c_char_p, _I64, _D]),
    "dgswe_batch_create": (C.c_int, [C.POINTER(Params), _P, C.c_int64, C.POINTER(_P)]),
    "dgswe_batch_destroy": (C.c_int, [_P]),
    "dgswe_batch_add": (C.c_int, [_P, _P, C.c_int64, _I]),
    "dgswe_batch_step": (C.c_int, [_P, C.c_int64]),
    "dgswe_batch_poll": (C.c_int, [_P, _I, C.c_int32, _I]),
    "dgswe_batch_retire": (C.c_int, [_P, C.c_int32]),
    "dgswe_batch_read": (C.c_int, [_P, C.c_int32, C.c_int, _D, C.POINTER(Mass)]),
    "dgswe_batch_info": (C.c_int, [_P, _I, _I64]),
    "dgswe_stream_probe": (C.c_int, [C.c_int32, C.c_int64, C.c_int32, _D]),
    "dgswe_last_error": (C.c_char_p, []),
}


def _load():
    try:  # share one HIP runtime with torch when torch is present
        import torch  # noqa: F401
    except Exception:  # pragma: no cover
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_14302_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def check(rc, func="dgswe"):
    if rc < 0:
        raise DgsweError(rc, func, lib.dgswe_last_error().decode())
    return rc


def call(name, *args):
    return check(getattr(lib, name)(*args), name)


def dptr(a):
    return a.ctypes.data_as(_D)


def fptr(a):
    return a.ctypes.data_as(_F)


def iptr(a):
    return a.ctypes.data_as(_I)
