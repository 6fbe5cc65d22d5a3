"""MI355X-native (gfx950) force-and-integrate loop of the bonded-particle model
for magneto-elastic rods: HIP kernels behind the C ABI of include/rod.h, with a
thin ctypes binding. PyTorch only supplies device memory and streams."""
from ._lib import (LIB_PATH, ROD_FP64, ROD_MIXED, RodError, TERM_ALL, TERM_BOND, TERM_CONTACT,
                   TERM_DAMP, TERM_DIPOLE, TERM_EXT, TERM_ZEEMAN, load)
from .sim import RodSim, rod_energy, rod_free, rod_grad, rod_init, rod_step, rod_trajectory
from .lbm import Lattice

__all__ = ["RodSim", "Lattice", "RodError", "rod_trajectory", "rod_init", "rod_step", "rod_energy", "rod_grad", "rod_free",
           "load", "LIB_PATH", "ROD_FP64", "ROD_MIXED", "TERM_ALL", "TERM_BOND", "TERM_CONTACT",
           "TERM_DAMP", "TERM_DIPOLE", "TERM_EXT", "TERM_ZEEMAN"]
