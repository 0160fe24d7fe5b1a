"""Forward model, observations and cost (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Physics.  The paper's constraint is 2D incompressible Navier-Stokes (Sec. II.A,
Eq. (1)); the forced case adds the body force f = (A sin(n_f y), 0) (Sec. III.E,
Eq. (24)).  This oracle integrates the same dynamics in vorticity form,

    d omega / dt = L omega + Nl(omega),
    L  = -(nu |k|^2 + mu)                       (viscosity and linear drag),
    Nl = -P(u d_x omega + v d_y omega) + P f_omega,
    f_omega = curl f = -A n_f cos(n_f y),

with the streamfunction psi = Psi omega (-Lap psi = omega), u = d_y psi,
v = -d_x psi.  P is the de-aliasing projector of the 2/3 rule: it keeps the
modes with |kx| <= Kc, |ky| <= Kc, k != 0, where Kc is the largest integer
below N/3 (square mask; zero mean).  The time scheme is the integrating-factor
(Lawson) fourth-order Runge-Kutta method: classical RK4 applied to
exp(-L t) omega.  The paper's own solver (fractional step, AB2/CN, Sec. III)
is not reproduced; this is the scheme the hot path implements.

Observation operator (Sec. II.A, Eqs. (2)-(3); Sec. II.C): velocity at grid
points (i s, j s) (stride s, offset 0) at a set of step indices.  The cost is
the plain Euclidean sum J = 1/2 sum_n sum_probes |u - m|^2 over both
components, no quadrature weights.
"""

from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from .dft import fft2, ifft2


@dataclass(frozen=True)
class Physics:
    N: int
    nu: float
    dt: float
    mu: float = 0.0            # linear drag
    forcing_amp: float = 0.0   # A in f = (A sin(n_f y), 0)
    forcing_k: int = 4         # n_f


class Grid:
    """Wavenumbers, de-aliasing mask and the velocity / derivative multipliers."""

    def __init__(self, N):
        self.N = N
        k = np.arange(N, dtype=np.int64)
        k[k >= N // 2] -= N
        self.kx = np.broadcast_to(k[None, :], (N, N)).astype(np.float64)
        self.ky = np.broadcast_to(k[:, None], (N, N)).astype(np.float64)
        self.ikx = np.broadcast_to(k[None, :], (N, N))
        self.iky = np.broadcast_to(k[:, None], (N, N))
        self.k2 = self.kx ** 2 + self.ky ** 2
        self.Kc = (N - 1) // 3
        self.mask = ((np.abs(self.ikx) <= self.Kc) & (np.abs(self.iky) <= self.Kc)
                     & (self.ikx ** 2 + self.iky ** 2 > 0)).astype(np.float64)
        with np.errstate(divide="ignore"):
            self.inv_k2 = np.where(self.mask > 0, 1.0 / np.where(self.k2 > 0, self.k2, 1.0), 0.0)
        # Operators on real fields, each composed with P:
        #   Psi : 1/k^2     U : i ky / k^2     V : -i kx / k^2
        #   Dx  : i kx      Dy : i ky
        self.m_psi = self.inv_k2
        self.m_u = 1j * self.ky * self.inv_k2
        self.m_v = -1j * self.kx * self.inv_k2
        self.m_dx = 1j * self.kx * self.mask
        self.m_dy = 1j * self.ky * self.mask
        j = np.arange(N)
        self.x = 2.0 * np.pi * j / N
        self.y = 2.0 * np.pi * j / N

    def apply(self, mult, f):
        """Real field f -> real(F^-1[mult F f])."""
        return np.real(ifft2(mult * fft2(f)))

    def to_phys(self, mult, fhat):
        """Spectrum -> real(F^-1[mult fhat])."""
        return np.real(ifft2(mult * fhat))


_GRIDS = {}


def grid(N):
    if N not in _GRIDS:
        _GRIDS[N] = Grid(N)
    return _GRIDS[N]


def forcing_hat(g, phys):
    """P F[f_omega] with f_omega = -A n_f cos(n_f y) (curl of Eq. (24)'s force)."""
    if phys.forcing_amp == 0.0:
        return np.zeros((g.N, g.N), dtype=np.complex128)
    fw = -phys.forcing_amp * phys.forcing_k * np.cos(phys.forcing_k * g.y)
    f = np.broadcast_to(fw[:, None], (g.N, g.N))
    return g.mask * fft2(f)


def lin_factor(g, phys, tau):
    """exp(L tau) with L = -(nu k^2 + mu), a real diagonal multiplier."""
    return np.exp(-(phys.nu * g.k2 + phys.mu) * tau)


def velocity_and_gradient(g, w_hat):
    """u, v, d_x omega, d_y omega in physical space from the spectrum of omega."""
    return (g.to_phys(g.m_u, w_hat), g.to_phys(g.m_v, w_hat),
            g.to_phys(g.m_dx, w_hat), g.to_phys(g.m_dy, w_hat))


def nonlinear(g, w_hat, f_hat):
    """Spectrum of Nl(omega) = -P(u omega_x + v omega_y) + P f_omega."""
    u, v, wx, wy = velocity_and_gradient(g, w_hat)
    return -g.mask * fft2(u * wx + v * wy) + f_hat


def lawson_step(g, phys, w_hat, f_hat, E1=None, E2=None):
    """One integrating-factor RK4 step; returns (w_next, (a, b, c, d), stages).

    a = Nl(w_n);             w_a = E(h/2)(w_n + h/2 a)
    b = Nl(w_a);             w_b = E(h/2) w_n + h/2 b
    c = Nl(w_b);             w_c = E(h) w_n + h E(h/2) c
    d = Nl(w_c)
    w_{n+1} = E(h) w_n + h/6 (E(h) a + 2 E(h/2)(b + c) + d)
    """
    h = phys.dt
    if E1 is None:
        E1 = lin_factor(g, phys, h)
        E2 = lin_factor(g, phys, 0.5 * h)
    a = nonlinear(g, w_hat, f_hat)
    wa = E2 * (w_hat + 0.5 * h * a)
    b = nonlinear(g, wa, f_hat)
    wb = E2 * w_hat + 0.5 * h * b
    c = nonlinear(g, wb, f_hat)
    wc = E1 * w_hat + h * E2 * c
    d = nonlinear(g, wc, f_hat)
    w_next = E1 * w_hat + (h / 6.0) * (E1 * a + 2.0 * E2 * (b + c) + d)
    return w_next, (w_hat, wa, wb, wc)


@dataclass
class Obs:
    """Observation set: probe stride, step indices and (optional) values.

    values has shape [n_times][2][M][M] (component 0 = u, 1 = v), M = N / stride,
    value [t][c][j][i] observed at grid point (x = i*stride, y = j*stride).
    """
    stride: int
    steps: Sequence[int]
    values: Optional[np.ndarray] = None


def observe(g, w_hat, stride):
    """Velocity at the probes: array [2][M][M]."""
    u = g.to_phys(g.m_u, w_hat)
    v = g.to_phys(g.m_v, w_hat)
    return np.stack([u[::stride, ::stride], v[::stride, ::stride]])


def initial_spectrum(g, omega0):
    """Trajectory start: P applied to the input field (spectrum)."""
    return g.mask * fft2(omega0)


def trajectory(omega0, phys, n_steps):
    """Spectra w_0..w_H of the trajectory from physical omega0."""
    g = grid(phys.N)
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    w = initial_spectrum(g, omega0)
    traj = [w]
    for _ in range(n_steps):
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
        traj.append(w)
    return traj


def sobolev_term(g, w0_hat, lam):
    """(lam/2) int |grad u0|^2 dOmega of Eq. (4) for the band-limited initial
    state: for a periodic divergence-free field int |grad u|^2 = int omega^2,
    and the grid rule (2 pi / N)^2 sum_ij omega_ij^2 is exact for it."""
    w = g.to_phys(1.0, w0_hat)
    return 0.5 * lam * (2.0 * np.pi / g.N) ** 2 * float(np.sum(w * w))


def forward(omega0, phys, n_steps, obs: Optional[Obs] = None, sobolev=0.0):
    """Run the forward model from a physical field.

    Returns (omega_T physical, J or None, model observations [n_t][2][M][M] or None).
    With sobolev = lambda > 0, J includes the regularisation term of Eq. (4).
    """
    g = grid(phys.N)
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    w = initial_spectrum(g, omega0)
    steps = list(obs.steps) if obs is not None else []
    model_obs = []
    J = 0.0

    def record(n, w):
        nonlocal J
        if n in steps:
            o = observe(g, w, obs.stride)
            model_obs.append(o)
            if obs.values is not None:
                r = o - obs.values[steps.index(n)]
                J += 0.5 * float(np.sum(r * r))

    if sobolev > 0.0 and obs is not None and obs.values is not None:
        J += sobolev_term(g, w, sobolev)
    record(0, w)
    for n in range(n_steps):
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
        record(n + 1, w)
    omega_T = g.to_phys(1.0, w)
    if obs is None:
        return omega_T, None, None
    return omega_T, (J if obs.values is not None else None), np.array(model_obs)
