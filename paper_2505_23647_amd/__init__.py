"""paper_2505_23647_amd - Shan-Chen extended-stencil lattice Boltzmann on AMD MI355X.

The compute lives in ``libscl.so`` (HIP kernels for gfx950 behind the C ABI of
``include/scl.h``); this package holds its ctypes binding, the build step, seeded input
recipes, stencil-weight design and the autograd wrapper of the adjoint.
"""
from ._lib import (SCL_D2Q9, SCL_D3Q19, SCL_FP16S_FP32, SCL_FP32, SCL_FP32_SHIFTED, SCL_FP64, SCL_PSI_CLASSIC,
                   SCL_PSI_EPS, SCL_PSI_EXP, SclError)
from .lattice import Lattice, set_allocator, use_torch_allocator, velocity_set

__all__ = ["Lattice", "velocity_set", "set_allocator", "use_torch_allocator", "SclError", "SCL_D2Q9", "SCL_D3Q19", "SCL_FP64", "SCL_FP32",
           "SCL_FP32_SHIFTED", "SCL_FP16S_FP32", "SCL_PSI_EXP", "SCL_PSI_EPS", "SCL_PSI_CLASSIC"]
