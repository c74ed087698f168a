"""mclbm on MI355X: the two-component pseudopotential lattice Boltzmann step of
arXiv:2009.12584 (Shan-Chen force, Guo forcing, half-way bounce-back, three
wetting rules) as hand-written HIP kernels behind a C ABI (include/mclbm.h).

This package holds the HIP sources (csrc/), their in-tree build, and a thin
ctypes binding.  Nothing here computes the method in Python.
"""
from .capi import (AVG_D2Q9, AVG_D2Q25, BC_LLKC, BC_MARTYS_CHEN, BC_VIRTUAL_IMPROVED, STORE_F16, STORE_F32,
                   LbmError)
from .sim import Batch, Pool, Simulation, mask_disk, mask_plane

__all__ = ["Simulation", "Batch", "Pool", "mask_plane", "mask_disk", "LbmError", "BC_MARTYS_CHEN", "BC_LLKC",
           "BC_VIRTUAL_IMPROVED", "AVG_D2Q25", "AVG_D2Q9", "STORE_F32", "STORE_F16"]
