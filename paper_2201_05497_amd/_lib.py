"""ctypes loader of liblmspdhg.so: argument and return types of every C ABI
entry point declared in include/lmspdhg.h.  There is no fallback: if the
library is not built, importing the package raises."""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblmspdhg.so")

LM_OK, LM_EINVAL, LM_ERANGE, LM_ENOMEM, LM_EHIP, LM_ESTATE = 0, -1, -2, -3, -4, -5
ERROR_NAMES = {LM_EINVAL: "LM_EINVAL", LM_ERANGE: "LM_ERANGE", LM_ENOMEM: "LM_ENOMEM",
               LM_EHIP: "LM_EHIP", LM_ESTATE: "LM_ESTATE"}


class LMGeom(ctypes.Structure):
    _fields_ = [("det", ctypes.c_void_p),
                ("n_cry", ctypes.c_int32), ("n_ring", ctypes.c_int32),
                ("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3),
                ("n_tof", ctypes.c_int32), ("tof_bin", ctypes.c_double),
                ("tof_fwhm", ctypes.c_double), ("tof_nsigma", ctypes.c_double),
                ("tof_on", ctypes.c_int32)]


# every exported symbol: name -> (restype, argtypes)
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
_GP = ctypes.POINTER(LMGeom)
SIGNATURES = {
    "lm_last_error": (ctypes.c_char_p, []),
    "lm_fwd": (ctypes.c_int, [_GP, _VP, _VP, _I64, _VP, _VP]),
    "lm_fwd_noalloc": (ctypes.c_int, [_GP, _VP, _VP, _I64, _VP, _VP]),
    "lm_back": (ctypes.c_int, [_GP, _VP, _VP, _I64, _VP, _VP]),
    "lm_sens": (ctypes.c_int, [_GP, _VP, _VP]),
    "lm_validate_events": (ctypes.c_int, [_GP, _VP, _I64, ctypes.POINTER(ctypes.c_int64), _VP]),
    "tv_grad": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), _VP, _VP, _VP]),
    "tv_div": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), _VP, _VP, _VP]),
    "lm_cost": (ctypes.c_int, [_GP, _VP, _VP, _VP, _I64, _VP, _D, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_double), _VP]),
    "lm_plan_bytes": (ctypes.c_int, [_GP, _I64, _I32, ctypes.POINTER(ctypes.c_size_t)]),
    "lm_plan_bytes_ex": (ctypes.c_int, [_GP, _I64, _I32, _I32, ctypes.POINTER(ctypes.c_size_t)]),
    "lm_plan_create": (ctypes.c_int, [_GP, _VP, _VP, _I64, _I32, _VP, _D, _D, _D, _D, _VP,
                                      ctypes.POINTER(_VP)]),
    "lm_spdhg_init": (ctypes.c_int, [_VP, _VP, _VP]),
    "lm_spdhg_epoch": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(ctypes.c_int32), _I32, _VP]),
    "lm_plan_set_prior_image": (ctypes.c_int, [_VP, _VP, _D, _VP]),
    "lm_plan_set_event_factors": (ctypes.c_int, [_VP, _VP, _VP]),
    "lm_plan_set_resolution": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), _VP]),
    "lm_plan_info": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int64)]),
    "lm_plan_get_lists": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    "lm_plan_get_layout": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lm_plan_get_images": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lm_plan_get_state": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_int64), _VP]),
    "lm_plan_set_state": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, _I64, _VP]),
    "lm_plan_timing": (ctypes.c_int, [_VP, ctypes.c_int]),
    "lm_plan_set_tracing": (ctypes.c_int, [_VP, ctypes.c_int]),
    "lm_plan_get_timing": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "lm_plan_destroy": (ctypes.c_int, [_VP]),
    "lm_emtv": (ctypes.c_int, [_GP, _VP, _VP, _I64, _I32, _I32, _VP, ctypes.c_float, _I32, _VP, _VP]),
}

_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python paper_2201_05497_amd/build.py` "
                "(the HIP library is required: there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LMError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = load().lm_last_error().decode(errors="replace")
        super().__init__(f"{where}: {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != LM_OK:
        raise LMError(code, where)
