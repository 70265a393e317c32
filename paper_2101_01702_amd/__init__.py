"""Reactive-mixture lattice Boltzmann step (Sawant, Dorschner & Karlin) on MI355X.

The hot path is a HIP library (liblbm.so, C ABI in include/lbm.h); this package holds
its Python binding (``lbm``), the build script (``build``) and seeded synthetic
workloads (``workloads``).
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "lbm", "build"]
