"""MI355X library for gauged (superposed) Gaussian fermionic PEPS Monte Carlo.

The compute path is libggf.so (HIP kernels for gfx950 behind the C ABI of
include/ggf.h); ``paper_2412_01737_amd.ggf`` is its thin Python binding.
Build with ``python -m paper_2412_01737_amd.build``.
"""
from . import ggf  # noqa: F401  (does not load the library until first use)

__all__ = ["ggf"]
