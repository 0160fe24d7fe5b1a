"""MI355X-native hot path of preconditioned adjoint data assimilation for 2D
turbulence (Ke, You & Wang, arXiv 2602.14016).

The computation lives in libpadjoint.so (HIP kernels for gfx950 behind the C
ABI of include/pa.h); this package only marshals arguments from PyTorch
tensors and streams.  Importing the package does not load the library;
constructing a Solver does, and fails loudly if it is missing.
"""

from .solver import (Solver, KernelSpec, Observations, IDENTITY, EXP_ABS, FRACTIONAL, HEAT, VELOCITY, VORTICITY,
                     STREAMFUNCTION)

__all__ = ["Solver", "KernelSpec", "Observations", "IDENTITY", "EXP_ABS", "FRACTIONAL", "HEAT",
           "VELOCITY", "VORTICITY", "STREAMFUNCTION"]
