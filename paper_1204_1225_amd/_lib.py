"""ctypes mirror of include/kirchhoff.h and the loader of libkirchhoff.so.

Argument marshalling only: every computation happens in the HIP library.
The library must have been built (paper_1204_1225_amd.build.build()); a
missing library raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# KM_LIBRARY names another build of this library (the sanitizer build of its
# host code, for instance); by default the in-tree one
LIB_PATH = os.environ.get("KM_LIBRARY") or os.path.join(HERE, "libkirchhoff.so")
ABI_VERSION = 4

KM_OK, KM_E_INVALID, KM_E_UNSUPPORTED, KM_E_HIP, KM_E_NOMEM = range(5)
KM_F32, KM_BF16, KM_F16 = 0, 1, 2
KM_W_UNIT, KM_W_COSCOS_OVER_TT = 0, 1
KM_TIME_FP32, KM_TIME_EXTENDED = 0, 1

_vp = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class KmTraces(ctypes.Structure):
    _fields_ = [("n_traces", _i64), ("n_samples", _i32), ("dtype", _i32), ("trace_stride", _i64),
                ("t_first", _f64), ("dt", _f64), ("data", _vp), ("scale", _vp), ("src", _vp), ("rec", _vp),
                ("bin", _vp)]


class KmGrid(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("nz", _i32), ("n_bins", _i32), ("x", _vp), ("y", _vp)]


class KmTraveltime(ctypes.Structure):
    _fields_ = [("t0sq", _vp), ("s2", _vp), ("r2", _vp), ("time_precision", _i32)]


class KmTtable(ctypes.Structure):
    _fields_ = [("n_h", _i32), ("dh", _f64), ("t", _vp), ("r2", _vp), ("time_precision", _i32), ("amp", _vp)]


class KmLtable(ctypes.Structure):
    _fields_ = [("n_h", _i32), ("dh", _f64), ("n_gx", _i32), ("n_gy", _i32), ("gx0", _f64), ("gy0", _f64),
                ("gdx", _f64), ("gdy", _f64), ("t", _vp), ("r2", _vp), ("time_precision", _i32), ("amp", _vp)]


class KmAntialias(ctypes.Structure):
    _fields_ = [("dx", _f64), ("dy", _f64), ("max_half", _i32)]


class KmWeight(ctypes.Structure):
    _fields_ = [("kind", _i32)]


class KmTileInfo(ctypes.Structure):
    _fields_ = [("waves", _i32), ("column_groups", _i32), ("depth_slots", _i32), ("lds_budget", _i32),
                ("trace_quads", _i32), ("shape", _i32), ("level", _i32), ("lds16", _i32)]


class KmProblem(ctypes.Structure):
    _fields_ = [("traces", KmTraces), ("grid", KmGrid), ("tt", KmTraveltime), ("weight", KmWeight),
                ("image", _vp)]


class KirchhoffError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"status {status}: {message}")
        self.status = status


_lib = None

# (name, restype, argtypes) for every entry point of include/kirchhoff.h
_P = ctypes.POINTER
SIGNATURES = {
    "km_abi_version": (ctypes.c_int, []),
    "km_last_error": (ctypes.c_char_p, []),
    "km_max_samples": (_i32, []),
    "kirchhoff_migrate": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmTraveltime), _P(KmWeight), _vp, _i32, _i32, _vp]),
    "kirchhoff_demigrate": (ctypes.c_int, [_vp, _P(KmGrid), _P(KmTraveltime), _P(KmWeight), _P(KmTraces), _i32, _i32, _vp]),
    "kirchhoff_migrate_table": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmTtable), _vp, _i32, _i32, _vp]),
    "kirchhoff_demigrate_table": (ctypes.c_int, [_vp, _P(KmGrid), _P(KmTtable), _P(KmTraces), _i32, _i32, _vp]),
    "kirchhoff_migrate_ltable": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmLtable), _vp, _i32, _i32, _vp]),
    "kirchhoff_demigrate_ltable": (ctypes.c_int, [_vp, _P(KmGrid), _P(KmLtable), _P(KmTraces), _i32, _i32, _vp]),
    "kirchhoff_migrate_aa": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmTraveltime), _P(KmWeight),
                                            _P(KmAntialias), _vp, _i32, _i32, _vp]),
    "kirchhoff_demigrate_aa": (ctypes.c_int, [_vp, _P(KmGrid), _P(KmTraveltime), _P(KmWeight), _P(KmAntialias),
                                              _P(KmTraces), _i32, _i32, _vp]),
    "km_count_contributions": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmTraveltime), _vp, _vp]),
    "km_count_contributions_host": (ctypes.c_int, [_P(KmTraces), _P(KmGrid), _P(KmTraveltime), _i32, _P(_i64),
                                                   _P(_i64)]),
    "km_dot_f64": (ctypes.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "km_axpby": (ctypes.c_int, [_f64, _vp, _f64, _vp, _i64, _vp]),
    "km_trace_filter": (ctypes.c_int, [_vp, _i64, _vp, _i64, _i64, _i32, _vp, _i32, _i32, _i32, _vp]),
    "km_stack_offsets": (ctypes.c_int, [_vp, _i32, _i64, _vp, _vp]),
    "km_cig_moveout": (ctypes.c_int, [_vp, _P(KmGrid), _vp, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp]),
    "km_tile_count": (_i32, [_i32]),
    "km_tile_levels": (_i32, [_i32]),
    "km_tile_describe": (ctypes.c_int, [_i32, _i32, _P(KmTileInfo)]),
    "km_tune": (ctypes.c_int, [_i32, _P(KmTraces), _P(KmGrid), _P(KmTraveltime), _P(KmWeight), _P(KmTtable),
                               _P(KmAntialias), _vp, _i32, _vp, _P(_i32), _P(ctypes.c_float)]),
    "km_tune_ltable": (ctypes.c_int, [_i32, _P(KmTraces), _P(KmGrid), _P(KmLtable), _vp, _i32, _vp,
                                       ctypes.POINTER(_i32), ctypes.POINTER(ctypes.c_float)]),
    "km_tune_lookup": (_i32, [_i32, _i32, _i32, _i32, _i32, _i32]),
    "km_tune_record": (ctypes.c_int, [_i32, _i32, _i32, _i32, _i32, _i32, _i32, ctypes.c_float]),
    "km_batch_create": (ctypes.c_int, [_P(KmProblem), _i32, _i32, _i32, _vp, _P(_vp)]),
    "km_batch_run": (ctypes.c_int, [_vp, _vp]),
    "km_batch_migrate_static": (ctypes.c_int, [_P(KmProblem), _i32, _i32, _vp]),
    "km_batch_info": (ctypes.c_int, [_vp, _P(_i64), _P(_i32)]),
    "km_batch_destroy": (ctypes.c_int, [_vp]),
    "km_probe_issue": (ctypes.c_int, [_i32, _i32, _i32, _vp, _P(ctypes.c_float)]),
}


def load():
    """Load libkirchhoff.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1204_1225_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.km_abi_version() != ABI_VERSION:
            raise RuntimeError(f"libkirchhoff ABI {lib.km_abi_version()} != {ABI_VERSION}")
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != KM_OK:
        raise KirchhoffError(status, load().km_last_error().decode(errors="replace"))
