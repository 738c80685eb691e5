"""ctypes binding of libscl.so (the C ABI declared in include/scl.h).

Argument marshalling only: every computation happens in the library's HIP kernels. The
binding never falls back to anything else; if the shared library is missing it raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscl.so")

SCL_OK, SCL_E_INVALID, SCL_E_NOMEM, SCL_E_DEVICE, SCL_E_STATE, SCL_E_NONFINITE, SCL_E_UNSUPPORTED = range(7)
SCL_D2Q9, SCL_D3Q19 = 0, 1
SCL_FP64, SCL_FP32, SCL_FP32_SHIFTED, SCL_FP16S_FP32 = 0, 1, 2, 3
SCL_PSI_EXP, SCL_PSI_EPS, SCL_PSI_CLASSIC = 0, 1, 2

STATUS_NAMES = {0: "SCL_OK", 1: "SCL_E_INVALID", 2: "SCL_E_NOMEM", 3: "SCL_E_DEVICE", 4: "SCL_E_STATE",
                5: "SCL_E_NONFINITE", 6: "SCL_E_UNSUPPORTED"}


class SclError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "scl_abi_version": (_I32, []),
    "scl_last_error": (ctypes.c_char_p, []),
    "scl_velocity_set": (_I32, [_I32, _P, _P]),
    "scl_set_allocator": (_I32, [_P, _P, _P]),
    "scl_create": (_I32, [_I32, _I32, _I32, _P, _P, ctypes.POINTER(_P)]),
    "scl_destroy": (_I32, [_P]),
    "scl_set_physics": (_I32, [_P, _P, _P, _I32, _P]),
    "scl_set_stencil": (_I32, [_P, _I32, _P, _P]),
    "scl_init_density": (_I32, [_P, _P, _I32]),
    "scl_step": (_I32, [_P, _I64]),
    "scl_step_timed": (_I32, [_P, _I64, ctypes.POINTER(_D)]),
    "scl_get_step_count": (_I32, [_P, ctypes.POINTER(_I64)]),
    "scl_get_density": (_I32, [_P, _P, _I32]),
    "scl_get_velocity": (_I32, [_P, _P, _I32]),
    "scl_get_force": (_I32, [_P, _P, _I32]),
    "scl_get_populations": (_I32, [_P, _P, _I32]),
    "scl_set_populations": (_I32, [_P, _P, _I32]),
    "scl_reduce_conserved": (_I32, [_P, _P, _P]),
    "scl_get_pressure_tensor": (_I32, [_P, _P, _I32]),
    "scl_droplet_observables": (_I32, [_P, _P, _P, _P]),
    "scl_flat_observables": (_I32, [_P, _P, _P]),
    "scl_set_force_squared": (_I32, [_P, _P]),
    "scl_set_tiling": (_I32, [_P, _I32, _I32, _I32]),
    "scl_get_tiling": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "scl_tune": (_I32, [_P, ctypes.c_char_p]),
    "scl_set_graph_steps": (_I32, [_P, _I32]),
    "scl_checkpointed_forward": (_I32, [_P, _I64, _I32]),
    "scl_adjoint": (_I32, [_P, _P, _P, _P, _P]),
    "scl_get_adjoint_populations": (_I32, [_P, _P, _I32]),
    "scl_droplet_observables_vjp": (_I32, [_P, _P, _P, _P, _P, _I32, _P, _P]),
}


def lib():
    """Load libscl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_23647_amd.build.build()")
        # torch brings its own copy of the HIP runtime. Loaded first, it also serves the
        # library; loaded after the library had initialised the system runtime, it finds no GPU.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != SCL_OK:
        raise SclError(status, lib().scl_last_error().decode())
    return status
