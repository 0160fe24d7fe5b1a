"""Tangent-linear model and discrete adjoint of the Lawson RK4 scheme (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

The paper derives the continuous adjoint (Sec. II.A, Eqs. (7)-(11): backward
equation with terminal condition zero and source M^T(M u - m)) and implements
a discrete adjoint obtained by summation by parts, exact to machine precision
(Sec. III).  The oracle follows the same principle for its own scheme:
discretise, then transpose.  Every real linear map F^-1[m F .] on the grid has
the transpose F^-1[conj(m) F .] for the grid (Euclidean) inner product, so
  P, Psi, E(tau)  are symmetric,
  U^T <-> conj(i ky / k^2),  V^T <-> conj(-i kx / k^2),
  Dx^T <-> conj(i kx),       Dy^T <-> conj(i ky),
and multiplication by a fixed field is symmetric.

Tangent of the right-hand side:
  Nl'(w) d = -P[(U d) w_x + u (Dx d) + (V d) w_y + v (Dy d)]
Its transpose, with Lam = P lam:
  Nl'(w)^T lam = -[U^T(w_x Lam) + Dx^T(u Lam) + V^T(w_y Lam) + Dy^T(v Lam)]

The gradient returned is dJ/d omega0 for the grid-Euclidean inner product
(the paper's gradient u0^dagger of Eq. (12) in this discretisation).
"""

import numpy as np

from .dft import fft2
from .model import (grid, forcing_hat, lin_factor, lawson_step, observe,
                    initial_spectrum, velocity_and_gradient, Obs, sobolev_term)


def nl_tangent(g, w_hat, d_hat):
    """Spectrum of Nl'(w) d."""
    u, v, wx, wy = velocity_and_gradient(g, w_hat)
    du, dv, dwx, dwy = velocity_and_gradient(g, d_hat)
    return -g.mask * fft2(du * wx + u * dwx + dv * wy + v * dwy)


def nl_adjoint(g, w_hat, lam_hat):
    """Spectrum of Nl'(w)^T lam (lam given by its spectrum)."""
    u, v, wx, wy = velocity_and_gradient(g, w_hat)
    Lam = g.to_phys(g.mask, lam_hat)
    return -(np.conj(g.m_u) * fft2(wx * Lam) + np.conj(g.m_dx) * fft2(u * Lam)
             + np.conj(g.m_v) * fft2(wy * Lam) + np.conj(g.m_dy) * fft2(v * Lam))


def tlm_step(g, phys, w_hat, dw_hat, E1, E2):
    """Tangent of one Lawson step at w_n applied to dw_n (spectra)."""
    h = phys.dt
    _wn, (wn, wa, wb, wc) = lawson_step(g, phys, w_hat, forcing_hat(g, phys), E1, E2)
    da = nl_tangent(g, wn, dw_hat)
    dwa = E2 * (dw_hat + 0.5 * h * da)
    db = nl_tangent(g, wa, dwa)
    dwb = E2 * dw_hat + 0.5 * h * db
    dc = nl_tangent(g, wb, dwb)
    dwc = E1 * dw_hat + h * E2 * dc
    dd = nl_tangent(g, wc, dwc)
    return E1 * dw_hat + (h / 6.0) * (E1 * da + 2.0 * E2 * (db + dc) + dd)


def adjoint_step(g, phys, w_hat, lam_hat, E1, E2):
    """Transpose of the tangent of one Lawson step at w_n, applied to lam_{n+1}."""
    h = phys.dt
    _wn, (wn, wa, wb, wc) = lawson_step(g, phys, w_hat, forcing_hat(g, phys), E1, E2)
    # w_{n+1} = E1 w_n + h/6 (E1 a + 2 E2 b + 2 E2 c + d)
    wbar = E1 * lam_hat
    abar = (h / 6.0) * E1 * lam_hat
    bbar = (h / 3.0) * E2 * lam_hat
    cbar = (h / 3.0) * E2 * lam_hat
    dbar = (h / 6.0) * lam_hat
    # d = Nl(w_c),  w_c = E1 w_n + h E2 c
    wcbar = nl_adjoint(g, wc, dbar)
    wbar = wbar + E1 * wcbar
    cbar = cbar + h * E2 * wcbar
    # c = Nl(w_b),  w_b = E2 w_n + h/2 b
    wbbar = nl_adjoint(g, wb, cbar)
    wbar = wbar + E2 * wbbar
    bbar = bbar + 0.5 * h * wbbar
    # b = Nl(w_a),  w_a = E2 (w_n + h/2 a)
    wabar = nl_adjoint(g, wa, bbar)
    wbar = wbar + E2 * wabar
    abar = abar + 0.5 * h * E2 * wabar
    # a = Nl(w_n)
    wbar = wbar + nl_adjoint(g, wn, abar)
    return wbar


def obs_source(g, w_hat, stride, values):
    """Spectrum of U^T(S^T r_u) + V^T(S^T r_v), r = M u - m at one time."""
    o = observe(g, w_hat, stride)
    r = o - values
    N = g.N
    Su = np.zeros((N, N))
    Sv = np.zeros((N, N))
    Su[::stride, ::stride] = r[0]
    Sv[::stride, ::stride] = r[1]
    src = np.conj(g.m_u) * fft2(Su) + np.conj(g.m_v) * fft2(Sv)
    return src, 0.5 * float(np.sum(r * r))


def adjoint_gradient(omega0, phys, n_steps, obs: Obs, sobolev=0.0):
    """Return (J, dJ/d omega0) for the observation set obs (values required).

    With sobolev = lambda > 0 the cost carries the term of Eq. (4),
    (lambda/2) (2 pi / N)^2 sum_ij (P omega0)^2, whose gradient
    lambda (2 pi / N)^2 P omega0 is added."""
    g = grid(phys.N)
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    steps = list(obs.steps)
    # forward sweep, storing the whole trajectory (the oracle has no memory limit)
    w = initial_spectrum(g, omega0)
    traj = [w]
    for _ in range(n_steps):
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
        traj.append(w)
    J = 0.0
    lam = np.zeros((g.N, g.N), dtype=np.complex128)
    if n_steps in steps:
        src, j = obs_source(g, traj[n_steps], obs.stride, obs.values[steps.index(n_steps)])
        lam = lam + src
        J += j
    for n in range(n_steps - 1, -1, -1):
        lam = adjoint_step(g, phys, traj[n], lam, E1, E2)
        if n in steps:
            src, j = obs_source(g, traj[n], obs.stride, obs.values[steps.index(n)])
            lam = lam + src
            J += j
    # omega_0 = P omega0_in  =>  dJ/d omega0_in = P lam_0
    grad = g.to_phys(g.mask, lam)
    if sobolev > 0.0:
        J += sobolev_term(g, traj[0], sobolev)
        grad = grad + sobolev * (2.0 * np.pi / g.N) ** 2 * g.to_phys(1.0, traj[0])
    return J, grad


def tlm_trajectory(omega0, domega0, phys, n_steps):
    """Tangent of the map omega0 -> omega_H (physical in, physical out)."""
    g = grid(phys.N)
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    w = initial_spectrum(g, omega0)
    dw = initial_spectrum(g, domega0)
    for _ in range(n_steps):
        dw = tlm_step(g, phys, w, dw, E1, E2)
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
    return g.to_phys(1.0, dw)


def adjoint_trajectory(omega0, mu_H, phys, n_steps):
    """Transpose of tlm_trajectory applied to a physical field mu_H."""
    g = grid(phys.N)
    traj = []
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    w = initial_spectrum(g, omega0)
    for _ in range(n_steps):
        traj.append(w)
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
    # omega_H (physical) = real F^-1 w_H: its transpose maps mu_H to F mu_H
    lam = fft2(mu_H)
    for n in range(n_steps - 1, -1, -1):
        lam = adjoint_step(g, phys, traj[n], lam, E1, E2)
    return g.to_phys(g.mask, lam)
