"""Seeded synthetic input generators (shapes and workloads).

Shared by the oracle tests, the GPU tests and the benchmark.  This package
only synthesises inputs; it holds none of the interpolation method's steps.
"""
from . import configs, shapes  # noqa: F401
