"""MI355X (gfx950) Matching Pursuit decoder.

The decoder itself is ``libmp.so`` (HIP kernels + the C ABI of
``include/mp.h``); :mod:`paper_0809_1833_amd.mp` is its Python binding.
Build with ``python -m paper_0809_1833_amd.build``.
"""
__all__ = ["mp", "build"]
