"""Learned-preconditioner PCG on AMD MI355X (gfx950).

The compute path is the HIP library liblpcg.so (C ABI in include/lpcg.h);
`paper_2305_16432_amd.lpcg` is its thin binding.  See that module.
"""
from . import lpcg  # noqa: F401

__all__ = ["lpcg"]
