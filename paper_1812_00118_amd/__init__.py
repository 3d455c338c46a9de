"""Phase-field lattice Boltzmann on AMD MI355X (gfx950).

Thin Python binding of the C-ABI library libpflb.so (include/pflb.h): argument
marshalling only.  Every step of the method runs in the library's HIP kernels;
PyTorch provides device memory and the current stream.  There is no CPU fallback:
if the library is missing or no GPU is present, the calls raise.
"""
from ._lib import (PflbError, Params, lib, load_library, STORE_FP32, STORE_FP16S,
                   STORE_FP32_INPLACE, BC_PERIODIC, BC_WALL)
from .sim import Sim, default_scales

__all__ = ["Sim", "Params", "PflbError", "lib", "load_library", "default_scales",
           "STORE_FP32", "STORE_FP16S", "STORE_FP32_INPLACE", "BC_PERIODIC", "BC_WALL"]
