"""MI355X (gfx950) coupled lattice Boltzmann - Langevin sweep for model H.

The compute path is the HIP library liblbl.so behind the C ABI of
include/lbl.h; ``paper_1104_0078_amd.lbl`` is its Python binding.
"""
from . import lbl  # noqa: F401

__all__ = ["lbl"]
