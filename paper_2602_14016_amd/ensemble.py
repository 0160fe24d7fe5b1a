"""Ensemble adjoint impulse response and per-shell backward growth rates (Sec. IV).

An ensemble of realizations sharing one initial spectrum (random phases,
seeds 0..B-1) is advanced forward and the adjoint is integrated backward from
a unit u-impulse at one grid point at the final time, all members in one
batched solve.  After every adjoint step the shell energies
sum_{k<=|k|<k+1} 1/2 |k|^2 |lambda_hat|^2 / N^4 are recorded per member; the
member mean gives E(k, tau) and its least-squares log-slope over the window
after the initial transient gives the growth rate of each shell.

statistics() runs large ensembles (the paper uses 3000 realizations) in
batches and reports, per backward step, the energy of the ensemble-mean
adjoint, the mean adjoint energy and their ratio (signal-to-noise), per
shell and in total, with the same quantities at growing subset sizes.
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


@dataclass
class EnsembleStats:
    members: int
    tau: torch.Tensor            # [rows], backward time of each row
    mean_energy: torch.Tensor    # [rows, n_shells]  mean over members of the shell energy
    energy_of_mean: torch.Tensor  # [rows, n_shells]  shell energy of the ensemble-mean adjoint
    total_mean: torch.Tensor     # [rows]  mean over members of the total adjoint energy
    total_of_mean: torch.Tensor  # [rows]  total energy of the ensemble-mean adjoint
    snr: torch.Tensor            # [rows]  total_of_mean / total_mean
    subsets: dict                # ensemble size -> {"total_mean", "total_of_mean", "snr"} at that size
    seconds: float


def statistics(N=256, members=3000, batch=64, n_steps=500, nu=1e-4, dt=2e-3, k0=10.0, n_shells=None,
               ckpt_every=None, impulse=None, subsets=(50, 100, 200, 400, 1000, 3000), seed0=0, tiles=None,
               verbose=False, mu=0.0, forcing_amp=0.0, forcing_k=4, init_kind=0, init_target=0.5, spinup=0):
    """Ensemble adjoint statistics of Sec. IV over `members` realizations (seeds
    seed0, seed0 + 1, ...), run in batches of at most `batch` members whose
    ends fall on every requested subset size.  The member sums are
    accumulated on the device in member order, so the statistics do not
    depend on the batch split; the statistics at each subset size are kept
    to show their convergence.

    Each realization starts from init_field(kind=init_kind, k0, init_target)
    of its seed, advanced `spinup` steps; with mu, forcing_amp and forcing_k
    the flow is the forced Kolmogorov flow (App. C: white noise, spin-up to
    the statistically stationary state)."""
    import time
    n_shells = n_shells or (N - 1) // 3
    ix, iy = impulse or (N // 2, N // 2)
    bounds = sorted({int(x) for x in subsets if 0 < x < members} | {members})
    solvers = {}

    def solver_for(b):
        if b not in solvers:
            sv = Solver(N, b, nu=nu, dt=dt, mu=mu, forcing_amp=forcing_amp, forcing_k=forcing_k)
            if tiles:
                sv.set_tiles(**tiles)
            solvers[b] = sv
        return solvers[b]

    main = solver_for(min(batch, members))
    acc = main.ensemble_accumulator(n_steps, n_shells)
    K = ckpt_every or main.fit_ckpt_every(n_steps)
    # One workspace, sized for the largest batch, serves every batch size in turn (batches run one
    # at a time): a whole-horizon tape fills most of the device, and reallocating it whenever the
    # batch size changes at a subset boundary would cost more than the solves.
    shared = main._ws if main._ws is not None and main._ws.numel() >= main.workspace_bytes(n_steps, K) + 256 \
        else None
    if shared is None:
        main._ws = None
        torch.cuda.empty_cache()
        shared = torch.empty(main.workspace_bytes(n_steps, K) + 256, dtype=torch.uint8, device=main.device)
    snaps = {}
    done = 0
    t0 = time.perf_counter()
    for end in bounds:
        while done < end:
            b = min(batch, end - done)
            sv = solver_for(b)
            sv._ws = shared
            w0 = sv.init_field(list(range(seed0 + done, seed0 + done + b)), kind=init_kind, k0=k0, target=init_target)
            if spinup:
                w0 = sv.forward(w0, spinup)["omega_T"]
            sv.adjoint_impulse(w0, n_steps, ix, iy, n_shells, ckpt_every=K, acc=acc)
            done += b
            if verbose:
                print(f"[ensemble] {done}/{members} members", flush=True)
        st = main.ensemble_stats(acc)
        snaps[end] = {k: st[k] for k in ("total_mean", "total_of_mean", "snr")}
    torch.cuda.synchronize(main.device)
    seconds = time.perf_counter() - t0
    tau = torch.arange(n_steps + 1, dtype=torch.float64, device=main.device) * dt
    return EnsembleStats(done, tau, st["mean_energy"], st["energy_of_mean"], st["total_mean"], st["total_of_mean"],
                         st["snr"], snaps, seconds)
