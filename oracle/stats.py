"""Turbulence statistics of a vorticity field (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The quantities the paper tabulates for its truth initial conditions (Sec. III,
Table 2), taken as grid means over the periodic box: u_rms (rms of one
velocity component), enstrophy Omega = <omega^2>/2, energy dissipation
eps = nu <|grad u|^2> with all four velocity derivatives formed separately,
enstrophy dissipation chi = nu <|grad omega|^2>, the Kraichnan wavenumber
k_eta = (chi / nu^3)^(1/6), the Taylor microscale lambda = u_rms / rms(du/dx)
(isotropic: rms(du/dx)^2 = <|grad u|^2>/4) and Re_lambda = u_rms lambda / nu,
Re_L = u_rms (2 pi) / nu.
"""

import math

import numpy as np

from .dft import fft2, ifft2
from .model import grid


def turbulence_statistics(omega, nu):
    N = omega.shape[0]
    g = grid(N)
    w_hat = g.mask * fft2(omega)
    u_hat, v_hat = g.m_u * w_hat, g.m_v * w_hat
    u, v = ifft2(u_hat).real, ifft2(v_hat).real
    grads_u = [ifft2(1j * d * f).real for f in (u_hat, v_hat) for d in (g.ikx, g.iky)]
    grads_w = [ifft2(1j * d * w_hat).real for d in (g.ikx, g.iky)]
    w = ifft2(w_hat).real
    u_rms = math.sqrt(float(np.mean(u * u + v * v)) / 2.0)
    omega_ens = 0.5 * float(np.mean(w * w))
    grad_u2 = float(sum(np.mean(q * q) for q in grads_u))
    eps = nu * grad_u2
    chi = nu * float(sum(np.mean(q * q) for q in grads_w))
    lam = u_rms / math.sqrt(grad_u2 / 4.0)
    return {"u_rms": u_rms, "Omega": omega_ens, "eps": eps, "chi": chi, "k_eta": (chi / nu ** 3) ** (1.0 / 6.0),
            "lambda": lam, "Re_lambda": u_rms * lam / nu, "Re_L": u_rms * 2.0 * math.pi / nu}
