"""MI355X non-negative tensor-train decomposition (nTT) by multiplicative updates.

The compute lives in libntt.so (HIP kernels for gfx950 behind the C ABI of
include/ntt.h); this package is its Python binding.
"""
from . import ntt  # noqa: F401
from .ntt import decompose, reconstruct, rel_error, load  # noqa: F401

__all__ = ["ntt", "decompose", "reconstruct", "rel_error", "load"]
