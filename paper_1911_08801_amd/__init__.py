"""MI355X-native artificial-scattering S_N (as-S_N) explicit step.

The compute path is libasn.so (HIP kernels for gfx950 behind the C ABI in
include/asn.h); ``paper_1911_08801_amd.asn`` is its ctypes binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libasn.so")

__all__ = ["LIB_PATH"]
