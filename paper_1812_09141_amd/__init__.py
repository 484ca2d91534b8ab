"""MI355X-native verification phase of exact set-similarity joins.

The compute path lives in ``libssj.so`` (HIP kernels for gfx950 behind the C
ABI of include/ssj.h); ``paper_1812_09141_amd.ssj`` is its thin ctypes binding
and ``paper_1812_09141_amd.build`` compiles it.  Importing the package itself
loads nothing.
"""
__all__ = ["ssj", "build"]
