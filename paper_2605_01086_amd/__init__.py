"""MI355X-native FPTC batch decoder (HIP kernels for gfx950 behind a C ABI).

`fptc` is the ctypes binding of libfptc.so (names as in include/fptc.h);
`codec` holds device-side containers and the host encoder helpers.
"""
from . import fptc  # noqa: F401

__all__ = ["fptc"]
