"""MI355X-native sign(H_W) b by restarted multishift FOM with LR deflation.

The computation lives in libsignkrylov.so (hand-written HIP kernels for
gfx950 behind a C ABI, include/signkrylov.h); this package is its build
script and a thin ctypes binding over torch device tensors.
"""
from . import _lib  # noqa: F401

__all__ = ["api", "build", "_lib"]
