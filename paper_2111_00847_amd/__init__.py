"""MI355X (gfx950) implementation of the consistent and conservative
phase-field lattice Boltzmann method (Zhan, Chai & Shi, arXiv:2111.00847).

The method runs in liblbm.so (HIP kernels behind the C ABI of include/lbm.h);
this package only marshals arguments (``api``) and wraps a lattice in a small
class (``sim.Sim``).
"""
from . import api  # noqa: F401
from ._lib import LbmError, LbmParams, lib  # noqa: F401
