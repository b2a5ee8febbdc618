"""MI355X-native per-scan voxel mapping (G-VOM, arXiv 2109.13176).

The product is the C-ABI library ``libgvom.so`` (include/gvom.h) built from the
HIP sources in ``csrc/``; ``gvom`` is its thin ctypes binding.
"""
from . import gvom  # noqa: F401
from .gvom import VoxelMap  # noqa: F401
