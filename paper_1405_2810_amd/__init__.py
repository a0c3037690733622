"""MI355X (gfx950) implementation of the online step of the Localized Reduced
Basis Multiscale method for two-phase flow (arXiv:1405.2810).

The compute path is the HIP library ``liblrbms.so`` (C ABI in
include/lrbms.h); ``paper_1405_2810_amd.lrbms`` is its ctypes binding.
"""
from . import lrbms  # noqa: F401  (the shared library itself loads on first use)

__all__ = ["lrbms"]
