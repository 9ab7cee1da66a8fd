"""ctypes loader for libsdc_mi355x.so (argument marshalling only; all compute is in HIP)."""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdc_mi355x.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sdc.h")

SDC_OK, SDC_EINVAL, SDC_ENOMEM, SDC_EHIP, SDC_ENONFINITE, SDC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16x3": 2}
QDELTAS = {"flex": 0, "ns": 1, "iepar": 2}
KERNEL_CLASSES = {"synthesis": 0, "grid": 1, "analysis": 2, "update": 3}
_NAMES = {0: "SDC_OK", -1: "SDC_EINVAL", -2: "SDC_ENOMEM", -3: "SDC_EHIP", -4: "SDC_ENONFINITE",
          -5: "SDC_EUNSUPPORTED"}

c_int, c_double, c_void_p, c_ll = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong
P_DOUBLE = ctypes.POINTER(ctypes.c_double)


class SdcConfig(ctypes.Structure):
    _fields_ = [("T", c_int), ("nlat", c_int), ("nlon", c_int),
                ("radius", c_double), ("gravity", c_double), ("omega", c_double), ("mean_depth", c_double),
                ("M", c_int), ("K", c_int), ("nodes", c_int), ("qdelta", c_int), ("precision", c_int),
                ("batch", c_int), ("implicit_coriolis", c_int)]


class SdcInfo(ctypes.Structure):
    _fields_ = [("T", c_int), ("nlat", c_int), ("nlon", c_int), ("ncoef", c_int), ("M", c_int),
                ("K", c_int), ("batch", c_int), ("precision", c_int),
                ("device_bytes", c_ll), ("table_bytes", c_ll)]


class SdcPlan(ctypes.Structure):
    _fields_ = [("syn_lat_tiles", c_int), ("syn_depth", c_int), ("ana_depth", c_int),
                ("ana_interleave", c_int), ("fuse_update", c_int),
                ("syn_recur", c_int), ("ana_recur", c_int), ("node_launch", c_int)]


class SDCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


_SIGS = {
    "sdc_init": (c_int, [ctypes.POINTER(SdcConfig), c_void_p, ctypes.POINTER(c_void_p)]),
    "sdc_free": (c_int, [c_void_p]),
    "sdc_step": (c_int, [c_void_p, c_void_p, c_double, c_int, c_int]),
    "sdc_step_graph": (c_int, [c_void_p, c_void_p, c_double, c_int, c_int]),
    "sdc_step_adjoint": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_int]),
    "imex2_step": (c_int, [c_void_p, c_void_p, c_double]),
    "sdc_tape_size": (c_int, [c_void_p, c_int, c_int, ctypes.POINTER(c_ll)]),
    "sdc_step_taped": (c_int, [c_void_p, c_void_p, c_double, c_int, c_int, c_void_p]),
    "sdc_step_adjoint_taped": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_int, c_int]),
    "sdc_step_sequential": (c_int, [c_void_p, c_void_p, c_double, c_int, c_int]),
    "sdc_step_sequential_graph": (c_int, [c_void_p, c_void_p, c_double, c_int, c_int]),
    "imex2_step_graph": (c_int, [c_void_p, c_void_p, c_double]),
    "imex2_step_noalloc": (c_int, [c_void_p, c_void_p, c_double]),
    "sdc_group_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_void_p, ctypes.POINTER(c_void_p)]),
    "sdc_group_step": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_double), c_int, c_int]),
    "sdc_group_sync": (c_int, [c_void_p]),
    "sdc_group_set_mode": (c_int, [c_void_p, c_int]),
    "sdc_group_get_mode": (c_int, [c_void_p, ctypes.POINTER(c_int)]),
    "sdc_group_autotune": (c_int, [c_void_p, ctypes.POINTER(c_void_p), ctypes.POINTER(c_double), c_int, c_int,
                                   c_int, ctypes.POINTER(c_int)]),
    "sdc_group_free": (c_int, [c_void_p]),
    "sht_forward": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sht_inverse": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sht_inverse_adjoint": (c_int, [c_void_p, c_void_p, c_void_p]),
    "imex_solve": (c_int, [c_void_p, c_double, c_void_p, c_void_p]),
    "eval_explicit": (c_int, [c_void_p, c_void_p, c_void_p]),
    "eval_implicit": (c_int, [c_void_p, c_void_p, c_void_p]),
    "sdc_sync": (c_int, [c_void_p]),
    "sdc_get_info": (c_int, [c_void_p, ctypes.POINTER(SdcInfo)]),
    "sdc_get_plan": (c_int, [c_void_p, ctypes.POINTER(SdcPlan)]),
    "sdc_set_plan": (c_int, [c_void_p, ctypes.POINTER(SdcPlan)]),
    "sdc_get_plan_for": (c_int, [c_void_p, c_int, ctypes.POINTER(SdcPlan)]),
    "sdc_set_plan_for": (c_int, [c_void_p, c_int, ctypes.POINTER(SdcPlan)]),
    "sdc_autotune": (c_int, [c_void_p, c_int, ctypes.POINTER(SdcPlan)]),
    "sdc_copy_grid": (c_int, [c_void_p, P_DOUBLE, P_DOUBLE]),
    "sdc_copy_coefficients": (c_int, [c_void_p, c_int, P_DOUBLE, P_DOUBLE]),
    "sdc_copy_legendre": (c_int, [c_void_p, c_int, P_DOUBLE, P_DOUBLE]),
    "sdc_timing_enable": (c_int, [c_void_p, c_int]),
    "sdc_debug_poison": (c_int, [c_void_p, c_int]),
    "sdc_timing_read": (c_int, [c_void_p, c_int, P_DOUBLE, ctypes.POINTER(c_ll)]),
    "sdc_last_error": (ctypes.c_char_p, []),
}

_lib = None


def header_functions():
    """Names of the functions declared in include/sdc.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def load():
    """Load the built library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != SDC_OK:
        msg = load().sdc_last_error().decode(errors="replace")
        raise SDCError(rc, msg)
