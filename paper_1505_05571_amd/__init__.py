"""Exact binary64 summation on MI355X (small and large superaccumulators).

The arithmetic runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in ``include/exsum.h``; ``paper_1505_05571_amd.api`` is a thin
ctypes binding to that library (argument marshalling only).
"""
from .api import *  # noqa: F401,F403
