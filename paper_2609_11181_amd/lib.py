"""ctypes binding of libsmartap.so: one Python function per C entry point,
same names, argument marshalling only. Raises if the library is missing."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmartap.so")

# enums of include/smartap.h
OK, EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED, EINTERNAL = 0, -1, -2, -3, -4, -5
FILTER_POLY, FILTER_TANH, FILTER_TABLE = 0, 1, 2
VAR_GALAXY, VAR_PIXEL, VAR_GALAXY_POSB = 0, 1, 2
PREC_FP64, PREC_FP32_GEO64, PREC_BF16X3, PREC_FP32_OUT64 = 0, 1, 2, 3
NORM_SUMMED_CAP, NORM_SUMMED_PIXCOUNT, NORM_RAW, NORM_AVERAGED = 0, 1, 2, 3
GAL_LANE, GAL_WAVE = 0, 1

EXPORTS = [
    "smart_init", "smart_finalize", "smart_last_error", "smart_version", "smart_filter_define",
    "smart_filter_table", "smart_filter_pieces", "smart_bin_galaxies", "smart_pixel_map", "smart_data_info", "smart_data_sources",
    "smart_data_export", "smart_barycentre_map",
    "smart_data_free", "smart_plan_create", "smart_run", "smart_last_pairs", "smart_plan_free",
    "smart_noise_batch", "smart_noise_angles", "smart_noise_seeded", "smart_noise_galaxy_batch",
    "smart_noise_galaxy_angles", "smart_noise_galaxy_seeded", "smart_mixed_batch", "smart_mixed_batch_noalloc", "smart_detect_peaks", "smart_plan_tiles",
    "smart_plan_set_timing", "smart_plan_kernel_ms", "smart_autotune", "smart_plan_galaxy_form",
    "smart_plan_set_galaxy_form",
]


class SmartError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"smartap error {code}: {msg}")
        self.code = code


_vp = C.c_void_p
_i64 = C.c_int64
_int = C.c_int

_SIGS = {
    "smart_init": (_int, [_int, C.POINTER(_vp)]),
    "smart_finalize": (None, [_vp]),
    "smart_last_error": (C.c_char_p, []),
    "smart_version": (C.c_char_p, []),
    "smart_filter_define": (_int, [_vp, _int, C.POINTER(C.c_double), _int, C.POINTER(_int)]),
    "smart_filter_table": (_int, [_vp, _int, C.POINTER(C.c_float), C.POINTER(_int)]),
    "smart_filter_pieces": (_int, [_vp, _int, C.c_double, C.POINTER(C.c_double), C.POINTER(_int)]),
    "smart_bin_galaxies": (_int, [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _int, _int, _vp, C.POINTER(_vp)]),
    "smart_pixel_map": (_int, [_vp, _int, _i64, _vp, _vp, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "smart_data_info": (_int, [_vp, C.POINTER(_i64), C.POINTER(_int), C.POINTER(_i64), C.POINTER(_i64),
                               C.POINTER(C.c_double)]),
    "smart_data_sources": (_int, [_vp, C.POINTER(_i64), _vp, _vp]),
    "smart_data_export": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "smart_data_free": (None, [_vp]),
    "smart_plan_create": (_int, [_vp, _vp, _int, _int, _i64, _vp, _int, C.POINTER(C.c_double),
                                 C.POINTER(_int), _int, _vp, C.POINTER(_vp)]),
    "smart_run": (_int, [_vp, _int, _vp, _vp]),
    "smart_last_pairs": (_int, [_vp, _vp, C.POINTER(C.c_double)]),
    "smart_plan_free": (None, [_vp]),
    "smart_noise_batch": (_int, [_vp, _vp, _int, _int, _int, _vp, _vp]),
    "smart_noise_galaxy_batch": (_int, [_vp, _vp, _int, _int, _vp, _vp]),
    "smart_noise_angles": (_int, [_vp, C.c_uint64, _i64, _int, _i64, _vp, _vp]),
    "smart_noise_seeded": (_int, [_vp, C.c_uint64, _i64, _int, _int, _int, _int, _vp, _vp]),
    "smart_noise_galaxy_angles": (_int, [_vp, C.c_uint64, _i64, _int, _i64, _vp, _vp]),
    "smart_noise_galaxy_seeded": (_int, [_vp, C.c_uint64, _i64, _int, _int, _int, _vp, _vp]),
    "smart_barycentre_map": (_int, [_vp, _vp, _vp]),
    "smart_mixed_batch": (_int, [_vp, _int, C.POINTER(_vp), C.POINTER(_int), C.POINTER(_vp), _vp]),
    "smart_mixed_batch_noalloc": (_int, [_vp, _int, C.POINTER(_vp), C.POINTER(_int), C.POINTER(_vp), _vp]),
    "smart_detect_peaks": (_int, [_vp, _int, _i64, _vp, _vp, _vp, C.c_double, _vp, C.POINTER(_i64), _vp]),
    "smart_plan_tiles": (_int, [_vp, _int, C.POINTER(_int), C.POINTER(_int), _vp, _vp, _vp]),
    "smart_plan_set_timing": (_int, [_vp, _int]),
    "smart_plan_galaxy_form": (_int, [_vp, _int, C.POINTER(_int)]),
    "smart_plan_set_galaxy_form": (_int, [_vp, _int, _int]),
    "smart_autotune": (_int, [_vp, _int, C.c_char_p, _vp]),
    "smart_plan_kernel_ms": (_int, [_vp, _int, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (no device work). Raises FileNotFoundError if
    it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: build it with `python -m paper_2609_11181_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(code: int):
    if code != OK:
        raise SmartError(code, load().smart_last_error().decode())
    return code


def get():
    """The loaded library (alias used by the tests)."""
    return load()
