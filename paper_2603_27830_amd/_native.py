"""ctypes binding of libsgp4mi.so (argument marshalling only).

Every computation runs in the library's HIP kernels; there is no fallback.
A missing or unloadable library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsgp4mi.so")

SGP4_FP64, SGP4_FP32, SGP4_FP32_MIXED = 0, 1, 2
PLAN_AUTOTUNE, PLAN_GRAPH = 1, 2
TEXT_FORMATS = {"tle": 1, "omm_kvn": 2, "omm_csv": 3, "omm_json": 4}
REC_CHECKSUM, REC_MISMATCH, REC_FIELD = 1, 2, 4
ERRORS = {0: "SGP4_OK", -1: "SGP4_E_ARG", -2: "SGP4_E_SIZE", -3: "SGP4_E_OFFSETS", -4: "SGP4_E_PRECISION",
          -5: "SGP4_E_HIP", -6: "SGP4_E_GRAVITY", -7: "SGP4_E_PLAN", -8: "SGP4_E_WORKSPACE",
          -9: "SGP4_E_HOST"}

# (name, restype, argtypes) for every symbol the public header declares.
_vp, _i64, _int, _dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
SIGNATURES = [
    ("sgp4_version", _int, []),
    ("sgp4_strerror", ctypes.c_char_p, [_int]),
    ("sgp4_consts_bytes", ctypes.c_size_t, [_i64]),
    ("sgp4_init", _int, [_dp, _i64, _vp, _vp, _vp, _vp]),
    ("sgp4_init_ex", _int, [_dp, _dp, _i64, _vp, _vp, _vp, _vp]),
    ("sgp4_propagate", _int, [_vp, _i64, _vp, _i64, _int, _vp, _vp, _vp, _vp]),
    ("sgp4_propagate_ex", _int, [_vp, _i64, _vp, _i64, _int, _vp, _vp, _vp, _int, _vp]),
    ("sgp4_propagate_elements", _int, [_dp, _i64, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                                       _vp]),
    ("sgp4_propagate_elements_ex", _int, [_dp, _dp, _i64, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp, _vp,
                                          ctypes.c_size_t, _vp]),
    ("sgp4_screen_workspace_bytes", ctypes.c_size_t, [_i64, _i64]),
    ("sgp4_screen", _int, [_vp, _int, _vp, _i64, _i64, ctypes.c_double, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t,
                           _vp]),
    ("sgp4_screen_ex", _int, [_vp, _int, _vp, _i64, _i64, ctypes.c_double, _i64, _vp, _vp, _vp, _vp,
                              ctypes.c_size_t, _int, _vp]),
    ("sgp4_screen_noalloc", _int, [_vp, _int, _vp, _i64, _i64, ctypes.c_double, _i64, _vp, _vp, _vp, _vp]),
    ("sgp4_text_count", _int, [ctypes.c_char_p, ctypes.c_size_t, _int, ctypes.POINTER(_i64)]),
    ("sgp4_text_parse", _int, [ctypes.c_char_p, ctypes.c_size_t, _int, _i64, _dp, _vp, _vp, _vp, _int]),
    ("sgp4_propagate_ragged", _int, [_vp, _i64, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp, _vp]),
    ("sgp4_plan_create", _int, [ctypes.POINTER(_vp), _vp, _i64, _vp, _vp, _i64, _int, _vp, _vp, _vp,
                                ctypes.c_uint, _vp]),
    ("sgp4_plan_create_config", _int, [ctypes.POINTER(_vp), _vp, _i64, _vp, _vp, _i64, _int, _vp, _vp, _vp,
                                       _int, _int, _int, ctypes.c_uint, _vp]),
    ("sgp4_plan_launch", _int, [_vp, _vp]),
    ("sgp4_plan_describe", _int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    ("sgp4_plan_destroy", None, [_vp]),
    ("sgp4_vjp", _int, [_i64, _vp, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp]),
    ("sgp4_vjp_ragged", _int, [_i64, _vp, _vp, _vp, _vp, _i64, _int, _vp, _vp, _vp, _vp]),
    ("sgp4_jacobian_ragged", _int, [_i64, _vp, _vp, _vp, _vp, _i64, _int, _vp, _vp]),
    ("sgp4_jacobian", _int, [_i64, _vp, _vp, _vp, _i64, _int, _vp, _vp]),
]

_LIB = None


class SGP4Error(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what} failed: {ERRORS.get(code, code)} ({strerror(code)})")


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsgp4mi.so not built at {LIB_PATH}: run __graft_entry__.build() "
                              "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def strerror(code: int) -> str:
    s = lib().sgp4_strerror(int(code))
    return s.decode() if s else ""


def check(code: int, what: str) -> None:
    if code != 0:
        raise SGP4Error(code, what)
