"""MI355X-native NLINV: the iteratively regularised Gauss-Newton reconstruction
of image and coil sensitivities (Schaetz & Uecker, Sec. 3), as hand-written
HIP kernels for gfx950 behind a C ABI (include/nlinv.h)."""
from . import _native
from .nlinv import FrameDims, Plan

__all__ = ["Plan", "FrameDims", "_native"]
