"""MI355X-native DDPS: domain-decomposing parallel sparse solver (hot path).

The solver itself lives in libddps.so (HIP kernels for gfx950 behind a C ABI,
include/ddps.h); `paper_1008_1700_amd.ddps` is its Python binding.
"""
__all__ = ["ddps", "build"]
