"""MI355X-native explicit finite-volume Euler residual and SSP-RK3 update.

The compute path lives in ``csrc/`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/fv.h``) and is reached from Python through
``paper_2305_18057_amd.fv``.  ``paper_2305_18057_amd.cases`` holds the seeded
synthetic input generators.  Importing this package loads nothing native.
"""
__all__ = ["cases", "fv"]
