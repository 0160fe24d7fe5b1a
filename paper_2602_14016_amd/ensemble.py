"""Ensemble adjoint impulse response and per-shell backward growth rates (Sec. IV).

An ensemble of realizations sharing one initial spectrum (random phases,
seeds 0..B-1) is advanced forward and the adjoint is integrated backward from
a unit u-impulse at one grid point at the final time, all members in one
batched solve.  After every adjoint step the shell energies
sum_{k<=|k|<k+1} 1/2 |k|^2 |lambda_hat|^2 / N^4 are recorded per member; the
member mean gives E(k, tau) and its least-squares log-slope over the window
after the initial transient gives the growth rate of each shell.
"""

from dataclasses import dataclass

import torch

from .solver import Solver


@dataclass
class EnsembleResult:
    shells: torch.Tensor      # [B, n_steps + 1, n_shells], row r = backward step r
    mean: torch.Tensor        # [n_steps + 1, n_shells]
    rates: torch.Tensor       # [n_shells]
    tau: torch.Tensor         # [n_steps + 1]


def run(N=256, members=64, n_steps=500, nu=1e-4, dt=2e-3, k0=10.0, n_shells=None, ckpt_every=50,
        impulse=None, tau_window=(0.3, 1.0), solver=None, omega0=None):
    s = solver or Solver(N, members, nu=nu, dt=dt)
    if omega0 is None:
        omega0 = s.init_field(list(range(members)), kind=0, k0=k0, target=0.5)
    n_shells = n_shells or (N - 1) // 3
    ix, iy = impulse or (N // 2, N // 2)
    shells, _ = s.adjoint_impulse(omega0, n_steps, ix, iy, n_shells, ckpt_every=ckpt_every)
    mean, rates = s.shell_growth(shells, *tau_window)
    tau = torch.arange(n_steps + 1, dtype=torch.float64, device=shells.device) * dt
    return EnsembleResult(shells, mean, rates, tau)
