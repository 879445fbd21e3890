"""MI355X-native quasi-Monte Carlo radiative transfer (Shulman, arXiv 2406.15632).

The hot path lives in libqrt.so (HIP kernels for gfx950 behind the C ABI of
include/qrt.h); paper_2406_15632_amd.qrt is its Python binding.
"""
__all__ = ["qrt", "build", "metrics"]
