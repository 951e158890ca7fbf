"""MI355X (gfx950) dense RGB-D alignment in inverse-depth parametrisation.

The method (Gutierrez-Gomez & Guerrero, RGBiD-SLAM, sec. 5.3, 6 and 7.2)
runs in hand-written HIP kernels behind the C ABI of ``include/rgbid.h``;
``paper_1807_08271_amd.rgbid`` is its ctypes binding.
"""
from . import rgbid  # noqa: F401

__all__ = ["rgbid"]
