"""MI355X-native matrix-free block-Jacobi PCG for periodic voxel elasticity.

The solver itself lives in the HIP/C++ shared library ``libelas3d.so``
(C-ABI declared in ``include/elas3d.h``); :mod:`.elas3d` is a thin ctypes
binding with the same entry-point names, and :mod:`.synth` makes seeded
synthetic inputs.
"""

__all__ = ["synth", "elas3d"]
