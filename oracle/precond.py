"""Weighting kernels, metric and the preconditioning operator (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper redefines the inner product with a symmetric positive convolution G
(Sec. II.B, Eqs. (13)-(16)); for a homogeneous G this is a real positive
Fourier multiplier Ghat(|k|).  The gradient in the new metric is the filtered
adjoint G u0^dagger (Eq. (17)).  Equivalently L-BFGS runs in the Euclidean
metric on the latent control s0 = G^{-1/2} u0, whose gradient is
G^{1/2} u0^dagger (Sec. II.C, Eqs. (18)-(19)).  Kernel families: algebraic
k^{-2 alpha} and heat-kernel exp(-nu beta k^2) with Ghat(0) = 1 (Sec. III.B);
the hot path also uses exp(-sigma |k|).

State and control here are vorticity fields.  The control metric multiplier
m(k)^2 is |k|^2 for the velocity metric (default: sum_x s^2 equals the
kinetic-energy norm sum_x |u|^2 when W = 1, so "identity" is the paper's
velocity control), 1 for the vorticity metric, or |k|^4 for the
streamfunction metric (sum_x s^2 = sum_x psi^2 when W = 1: the control
variables u0, omega0, psi0 of Sec. III.A).  precondition(f, p) is

    F^-1[ (m^2 W)^p 1_S F f ]

so omega0 = precondition(s, +1/2), s = precondition(omega0, -1/2), latent
gradient g_s = precondition(g_omega, +1/2), filtered gradient (Eq. (17)) is
precondition(g_omega, 1).  W = 1/k^2 in the velocity metric equals identity
in the vorticity metric (Sec. III.A, Eq. (21); Appendix B).
"""

from dataclasses import dataclass

import numpy as np

from .dft import fft2, ifft2
from .model import grid

IDENTITY, EXP_ABS, FRACTIONAL, HEAT = 0, 1, 2, 3
VELOCITY, VORTICITY, STREAMFUNCTION = 0, 1, 2


@dataclass(frozen=True)
class Kernel:
    kind: int = IDENTITY     # 0 identity, 1 exp(-param |k|), 2 |k|^(-2 param), 3 exp(-param |k|^2)
    param: float = 0.0
    metric: int = VELOCITY


def weight(g, kern: Kernel):
    """W(|k|) on the full grid, W(0) = 1."""
    kappa = np.sqrt(g.k2)
    pos = g.k2 > 0
    safe = np.where(pos, kappa, 1.0)
    if kern.kind == IDENTITY:
        W = np.ones_like(kappa)
    elif kern.kind == EXP_ABS:
        W = np.exp(-kern.param * kappa)
    elif kern.kind == FRACTIONAL:
        W = safe ** (-2.0 * kern.param)
    elif kern.kind == HEAT:
        W = np.exp(-kern.param * g.k2)
    else:
        raise ValueError("unknown kernel kind")
    return np.where(pos, W, 1.0)


def multiplier(g, kern: Kernel, power: float):
    """(m^2 W)^power on S, zero outside."""
    W = weight(g, kern)
    m2 = {VELOCITY: g.k2, VORTICITY: np.ones_like(g.k2), STREAMFUNCTION: g.k2 * g.k2}[kern.metric]
    base = np.where(g.mask > 0, m2 * W, 1.0)
    return np.where(g.mask > 0, base ** power, 0.0)


def precondition(f, kern: Kernel, power: float):
    """F^-1[(m^2 W)^power 1_S F f] for a physical field f (or batch)."""
    N = f.shape[-1]
    g = grid(N)
    return np.real(ifft2(multiplier(g, kern, power) * fft2(f)))
