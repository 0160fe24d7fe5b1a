"""CPU FP64 oracle for the preconditioned adjoint data-assimilation hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
(``paper_2602_14016_amd``) never does, and this package imports nothing from
it.  It shares no code, tables or constants with the HIP kernels.

Everything is NumPy in float64 / complex128.  Fourier transforms are this
package's own DFT (``oracle.dft``): explicit twiddle matrices applied with a
matrix product, no ``numpy.fft`` or ``scipy.fft``.

Paper: Ke, You & Wang, "Preconditioned Adjoint Data Assimilation for
Two-Dimensional Decaying and Forced Turbulence" (arXiv 2602.14016).

Modules
-------
dft        exact-twiddle DFT matrices and 2D transforms
model      grid, spectral operators, vorticity right-hand side, Lawson RK4,
           observations and cost (Sec. II.A, Eqs. (1)-(3); Eq. (24))
adjoint    tangent-linear and discrete adjoint of the scheme; gradient of J
           (Sec. II.A, Eqs. (11)-(12); Sec. III "summation by parts")
precond    weighting kernels W(k), metric, precondition (Sec. II.B-C,
           Eqs. (13)-(19); Sec. III.B)
optim      steepest descent and L-BFGS in the latent variable (Sec. II.C)
fields     counter-based RNG, initial fields, first guess (Sec. III)
ensemble   adjoint impulse response, shell energies, growth rates, ensemble statistics (Sec. IV)
checkpoint fewest recomputations that reverse a chain under a snapshot budget
stats      turbulence statistics of a field (Table 2 quantities)
"""

from .dft import twiddles, dft_matrix, fft2, ifft2
from .model import Physics, Grid, Obs, forward, trajectory, observe, nonlinear
from .adjoint import adjoint_gradient, tlm_step, adjoint_step, tlm_trajectory
from .precond import Kernel, weight, precondition
from .optim import lbfgs_two_loop, assimilate
from .fields import splitmix64, uniform01, init_field, first_guess
from .ensemble import impulse_adjoint, impulse_lambdas, shell_energy, total_energy, growth_rates, ensemble_statistics
from .checkpoint import min_advances, optimal_first_advances
from .stats import turbulence_statistics

__all__ = [
    "twiddles", "dft_matrix", "fft2", "ifft2",
    "Physics", "Grid", "Obs", "forward", "trajectory", "observe", "nonlinear",
    "adjoint_gradient", "tlm_step", "adjoint_step", "tlm_trajectory",
    "Kernel", "weight", "precondition",
    "lbfgs_two_loop", "assimilate",
    "splitmix64", "uniform01", "init_field", "first_guess",
    "impulse_adjoint", "impulse_lambdas", "shell_energy", "total_energy", "growth_rates",
    "ensemble_statistics", "min_advances", "optimal_first_advances", "turbulence_statistics",
]
