"""MI355X (gfx950) finite-temperature XL-BOMD hot path.

The computation lives in the HIP shared library _lib/libxlbomd.so behind the
C ABI declared in include/xlbomd.h; `binding` is a thin ctypes layer over it.
"""
from .binding import (XLBOMD, FP32, FP64, MIXED, MIXED_BF16X3, MIXED_BF16, Allocator,  # noqa: F401
                      TorchAllocator, XlbomdError, lib)
