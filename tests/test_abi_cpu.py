"""The C ABI library loads on the CPU host and exports what include/scl.h declares; host-side
argument validation that needs no device."""
import ctypes
import os
import re

import numpy as np

from paper_2505_23647_amd import _lib as B
from paper_2505_23647_amd.lattice import velocity_set
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "scl.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(scl_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    L = B.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
        assert n in B.SIGNATURES, n


def test_abi_version():
    assert B.lib().scl_abi_version() == 3


def test_velocity_sets_match_oracle_sets():
    for vs, d in ((B.SCL_D2Q9, 2), (B.SCL_D3Q19, 3)):
        xi, w = velocity_set(vs)
        oxi, ow = oracle.velset(d)
        lib_set = sorted((tuple(v), round(x, 15)) for v, x in zip(xi.tolist(), w))
        ora_set = sorted((tuple(v), round(x, 15)) for v, x in zip(oxi.tolist(), ow))
        assert lib_set == ora_set
    assert B.lib().scl_velocity_set(7, None, None) == -1


def test_create_rejects_bad_arguments_before_device_work():
    L = B.lib()
    h = ctypes.c_void_p()
    dims = np.array([16, 16, 1], dtype=np.int32)
    p = dims.ctypes.data_as(ctypes.c_void_p)
    assert L.scl_create(B.SCL_D2Q9, B.SCL_FP64, 0, p, None, ctypes.byref(h)) == B.SCL_E_INVALID
    assert L.scl_create(9, B.SCL_FP64, 1, p, None, ctypes.byref(h)) == B.SCL_E_INVALID
    assert L.scl_create(B.SCL_D2Q9, 11, 1, p, None, ctypes.byref(h)) == B.SCL_E_INVALID
    bad = np.array([16, 16, 2], dtype=np.int32)
    assert L.scl_create(B.SCL_D2Q9, B.SCL_FP64, 1, bad.ctypes.data_as(ctypes.c_void_p), None,
                        ctypes.byref(h)) == B.SCL_E_INVALID
    zero = np.array([16, 0, 1], dtype=np.int32)
    assert L.scl_create(B.SCL_D2Q9, B.SCL_FP64, 1, zero.ctypes.data_as(ctypes.c_void_p), None,
                        ctypes.byref(h)) == B.SCL_E_INVALID
    assert b"extent" in L.scl_last_error()
    assert L.scl_create(B.SCL_D2Q9, B.SCL_FP64, 1, p, None, None) == B.SCL_E_INVALID
    assert L.scl_destroy(None) == B.SCL_OK


def test_allocator_hook_arguments():
    """scl_set_allocator takes both functions or neither (no device work involved)."""
    from paper_2505_23647_amd import lattice
    a = lattice._ALLOC_T(lambda n, ctx, stream: None)
    assert B.lib().scl_set_allocator(ctypes.cast(a, ctypes.c_void_p), None, None) == B.SCL_E_INVALID
    assert B.lib().scl_set_allocator(None, None, None) == B.SCL_OK
