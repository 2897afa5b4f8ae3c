"""MI355X-native parallel bounding for permutation flow-shop branch-and-bound.

The compute path lives in ``libfsp.so`` (HIP kernels for gfx950 behind a C
ABI, declared in ``include/fsp.h``).  Importing this package loads nothing;
``paper_1206_4973_amd.fsp`` loads the library on first use and raises if it is
missing.
"""
__all__ = ["inputs", "fsp"]
