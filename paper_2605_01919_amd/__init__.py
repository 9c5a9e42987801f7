"""sdfi: consistent signed-distance interpolation on AMD MI355X (gfx950).

The compute path is the HIP library libsdfi.so (C ABI in include/sdfi.h);
``paper_2605_01919_amd.sdfi`` is its Python binding for torch GPU tensors.
"""
from . import sdfi  # noqa: F401
