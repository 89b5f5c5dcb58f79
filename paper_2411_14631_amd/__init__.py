"""MI355X-native octree MUSCL-Hancock / HLLC hydro step and uniform-level
PPCG Poisson solver (C ABI + HIP kernels).

The library lives in libry.so next to this file (built by build.py); the
Python binding in ry.py only marshals arguments.
"""
from .ry import BatchHydro, Hydro, Poisson, RyError, lib  # noqa: F401
