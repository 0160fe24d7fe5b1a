"""Adjoint impulse response, shell energies and backward growth rates (oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. IV of the paper: a unit perturbation of the u component at one point at
the final time T is propagated backward with the adjoint (the adjoint Green's
function); over an ensemble of forward realizations sharing one spectrum the
shell-wise adjoint energy is averaged.  The shell sum follows the isotropic
spectrum definition E(k) = sum_{k <= |k| < k+1} 1/2 |uhat|^2 (Sec. III,
Eq. (20), unit shell width).  The adjoint velocity is the curl of the adjoint
streamfunction-like field lambda: uhat = i ky lambda_hat, vhat = -i kx
lambda_hat, so the shell energy is sum 1/2 |k|^2 |lambda_hat|^2 / N^4.  Shell
membership uses the exact integer square root of kx^2 + ky^2.  The growth rate
of a shell is the least-squares slope of ln(mean energy) against backward time
tau after the initial transient (the paper reports about 0.3, Sec. IV).

Ensemble statistics (Sec. IV): the energy of the ensemble-mean adjoint (its
reproducible part), the mean over members of the adjoint energy (mean plus
fluctuations), per shell and in total, and their ratio, the signal-to-noise
ratio of the adjoint sensitivity.
"""

import math

import numpy as np

from .adjoint import adjoint_step
from .dft import fft2
from .model import grid, forcing_hat, lin_factor, lawson_step, initial_spectrum


def shell_index(g):
    """floor(|k|) from exact integer arithmetic."""
    m = (g.ikx ** 2 + g.iky ** 2).astype(np.int64)
    return np.vectorize(math.isqrt)(m)


def shell_energy(g, lam_hat, n_shells):
    """Shells k = 1..n_shells of sum 1/2 |k|^2 |lam_hat|^2 / N^4 over the full spectrum."""
    idx = shell_index(g)
    e = 0.5 * g.k2 * np.abs(lam_hat) ** 2 / float(g.N) ** 4
    out = np.zeros(n_shells)
    for k in range(1, n_shells + 1):
        out[k - 1] = float(np.sum(e[idx == k]))
    return out


def total_energy(g, lam_hat):
    """Adjoint velocity energy over the whole spectrum: sum 1/2 |k|^2 |lam_hat|^2 / N^4."""
    return float(np.sum(0.5 * g.k2 * np.abs(lam_hat) ** 2)) / float(g.N) ** 4


def impulse_lambdas(omega0, phys, n_steps, ix, iy):
    """Adjoint spectra lambda_hat (full N x N) of the impulse response, one per
    backward step (index 0 = terminal field, index r = step n_steps - r)."""
    g = grid(phys.N)
    fh = forcing_hat(g, phys)
    E1 = lin_factor(g, phys, phys.dt)
    E2 = lin_factor(g, phys, 0.5 * phys.dt)
    w = initial_spectrum(g, omega0)
    traj = []
    for _ in range(n_steps):
        traj.append(w)
        w, _st = lawson_step(g, phys, w, fh, E1, E2)
    e = np.zeros((g.N, g.N))
    e[iy, ix] = 1.0
    lam = np.conj(g.m_u) * fft2(e)
    out = [lam]
    for n in range(n_steps - 1, -1, -1):
        lam = adjoint_step(g, phys, traj[n], lam, E1, E2)
        out.append(lam)
    return out


def ensemble_statistics(omega0s, phys, n_steps, ix, iy, n_shells):
    """Ensemble adjoint statistics of Sec. IV over the members omega0s.

    Per backward step (rows as in impulse_adjoint):
      mean_energy[r][k-1]       mean over members of the shell energy,
      energy_of_mean[r][k-1]    shell energy of the ensemble-mean adjoint,
      total_mean_energy[r]      mean over members of the total adjoint energy,
      total_energy_of_mean[r]   total energy of the ensemble-mean adjoint,
      snr[r]                    total_energy_of_mean / total_mean_energy.
    """
    g = grid(phys.N)
    B = len(omega0s)
    lam_sum = None
    mean_e, tot_e = None, None
    for w0 in omega0s:
        lams = impulse_lambdas(w0, phys, n_steps, ix, iy)
        se = np.array([shell_energy(g, l, n_shells) for l in lams])
        te = np.array([total_energy(g, l) for l in lams])
        mean_e = se if mean_e is None else mean_e + se
        tot_e = te if tot_e is None else tot_e + te
        lam_sum = list(lams) if lam_sum is None else [a + l for a, l in zip(lam_sum, lams)]
    mean_lam = [l / B for l in lam_sum]
    eom = np.array([shell_energy(g, l, n_shells) for l in mean_lam])
    teom = np.array([total_energy(g, l) for l in mean_lam])
    tme = tot_e / B
    return {"mean_energy": mean_e / B, "energy_of_mean": eom, "total_mean_energy": tme,
            "total_energy_of_mean": teom, "snr": teom / tme}


def impulse_adjoint(omega0, phys, n_steps, ix, iy, n_shells):
    """Backward adjoint from a unit u-impulse at grid point (x = ix, y = iy) at the final step.

    Returns (shell energies [n_steps + 1][n_shells] indexed by backward step
    tau_n = (n_steps - n) dt, i.e. row 0 is the terminal field; gradient-like
    final field P lambda_0 (physical)).
    """
    g = grid(phys.N)
    lams = impulse_lambdas(omega0, phys, n_steps, ix, iy)
    return np.array([shell_energy(g, l, n_shells) for l in lams]), g.to_phys(g.mask, lams[-1])


def growth_rates(mean_energy, dt, tau_min=0.3, tau_max=1.0):
    """Least-squares slope of ln(mean shell energy) vs tau on [tau_min, tau_max].

    mean_energy[n][k] is indexed by backward step n (tau = n dt).
    """
    n = np.arange(mean_energy.shape[0])
    tau = n * dt
    sel = (tau >= tau_min - 1e-12) & (tau <= tau_max + 1e-12)
    t = tau[sel]
    out = np.full(mean_energy.shape[1], np.nan)
    if t.size < 2:
        return out
    tc = t - t.mean()
    for k in range(mean_energy.shape[1]):
        y = mean_energy[sel, k]
        if np.all(y > 0):
            ly = np.log(y)
            out[k] = float(np.sum(tc * (ly - ly.mean())) / np.sum(tc * tc))
    return out
