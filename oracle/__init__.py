"""CPU oracle of the periodic voxel elasticity solve (test infrastructure only).

A plain serial FP64 C implementation (``elas3d_oracle.c``) wrapped with
ctypes.  Only the tests, the smoke check and the benchmark's CPU-baseline
leg use it; the product library never imports it and shares no code with
it.  Every function follows a passage of ELAS3D-Xtal (arXiv 2602.07354),
cited in the C source.

Parity of every function here is pinned by ``tests/test_oracle_pins.py``
(closed forms, invariants, brute-force dense solves); none is unpinned.
"""

from .oracle import *  # noqa: F401,F403
from .oracle import __all__  # noqa: F401
