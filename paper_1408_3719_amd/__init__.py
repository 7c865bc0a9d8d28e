"""MI355X (gfx950) implementation of the cell-centred ALE ADER-WENO finite
volume scheme with time-accurate local time stepping on moving triangular
meshes (Boscheri, Dumbser, Zanotti, arXiv:1408.3719).

The numerics live in libaderweno.so (HIP kernels behind the C ABI of
include/aderweno.h); this package only marshals arguments.
"""
from .solver import Config, HostTopology, Solver
from ._lib import AderError, load

__all__ = ["Config", "Solver", "HostTopology", "AderError", "load"]
