"""Writes the oracle's expected values for the full-horizon GPU parity tests.

Run from the repository root:  python tests/golden/make_oracle_fixtures.py

It calls only the CPU oracle (oracle/) and NumPy; every input is generated
here from the oracle's seeded initial fields.  The GPU tests load the files
(numpy.load, no pickles) instead of spending minutes of CPU on the oracle:

  c1_full_horizon.npz   c1 at its full horizon: 256^2, nu = 1e-4, dt = 2e-3,
                        1000 steps, velocity probes at stride 8 at 5 evenly
                        spaced times from the truth of seed 0 (random phase,
                        k0 = 10, energy 0.5), initial field of seed 1:
                        observations, cost and gradient.
  ensemble_member17.npz the ensemble workload's member 17 (256^2, nu = 1e-4,
                        dt = 2e-3, seed 17, k0 = 10, energy 0.5): shell
                        energies |k| = 1..85 of the adjoint of a unit
                        u-impulse at (128, 128) after 500 steps, per backward
                        step.
  c2_100_steps.npz      the Kolmogorov configuration's physics on its grid
                        (512^2, nu = 1/40, drag 0.1, f_x = sin 4y, dt = 1e-3)
                        over a 100-step window: the field after 100 steps
                        from the random-phase field of seed 0 (k0 = 6,
                        energy 0.5), velocity probes at stride 16 at steps
                        0, 50, 100 from the field of seed 1, and the cost and
                        gradient at the seed-0 field.
  c1_grid_lbfgs.npz     L-BFGS at the differentiation configuration's grid and
                        physics (256^2, nu = 1e-4, dt = 2e-3) over a 50-step
                        window: probes at stride 8 at steps 0, 12, 25, 38, 50
                        from the truth of seed 0 (random phase, k0 = 10,
                        energy 0.5), the interpolated first guess from the
                        t = 0 probes, kernel exp(-0.05 |k|) in the velocity
                        metric, memory 10: the cost after each of 10
                        iterations and the estimates after 1, 5 and 10.
  c2_grid_lbfgs.npz     L-BFGS at the Kolmogorov configuration's grid and
                        physics (512^2, nu = 1/40, drag 0.1, f_x = sin 4y,
                        dt = 1e-3) over a 40-step window: probes at stride 16
                        at steps 0, 20, 40 from the random-phase field of
                        seed 1 (k0 = 6, energy 0.5), the interpolated first
                        guess from the t = 0 probes, kernel |k|^-1 in the
                        velocity metric, memory 10: the cost after each of 5
                        iterations and the estimates after 1, 3 and 5, kept at
                        every 2nd grid point in each direction (the first
                        guess in full).
  grid1024_50_steps.npz the largest grid (1024^2, nu = 1e-4, dt = 5e-4) over 50
                        steps from the random-phase field of seed 3 (k0 =
                        1024/25, energy 0.5): the field after 50 steps and the
                        cost and gradient of velocity probes at stride 16 at
                        steps 0, 25, 50 from the field of seed 4.  The field
                        and gradient are kept at every 4th grid point in each
                        direction (the tests compare those samples), the cost
                        in full.
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from oracle.model import Obs, Physics  # noqa: E402


def evenly_spaced(n_steps, n):
    return sorted({int(round(i * n_steps / (n - 1))) for i in range(n)})


def c1_full_horizon():
    N, H = 256, 1000
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    osteps = evenly_spaced(H, 5)
    truth = O.init_field(N, [0], kind=0, k0=10.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(8, osteps))
    w0 = O.init_field(N, [1], kind=0, k0=10.0, target=0.5)[0]
    J, g = O.adjoint_gradient(w0, ph, H, Obs(8, osteps, mo))
    np.savez(os.path.join(HERE, "c1_full_horizon.npz"), obs_steps=np.array(osteps), obs=np.asarray(mo),
             J=np.array(J), grad=g)


def ensemble_member17():
    N, H = 256, 500
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    w0 = O.init_field(N, [17], kind=0, k0=10.0, target=0.5)[0]
    rows = O.impulse_adjoint(w0, ph, H, N // 2, N // 2, 85)[0]
    np.savez(os.path.join(HERE, "ensemble_member17.npz"), shells=np.asarray(rows))


def c2_100_steps():
    N, H = 512, 100
    ph = Physics(N=N, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    osteps = [0, 50, 100]
    w0 = O.init_field(N, [0], kind=0, k0=6.0, target=0.5)[0]
    truth = O.init_field(N, [1], kind=0, k0=6.0, target=0.5)[0]
    omega_T = O.forward(w0, ph, H)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(16, osteps))
    J, g = O.adjoint_gradient(w0, ph, H, Obs(16, osteps, mo))
    np.savez(os.path.join(HERE, "c2_100_steps.npz"), obs_steps=np.array(osteps), obs=np.asarray(mo),
             omega_T=np.asarray(omega_T), J=np.array(J), grad=g)


def c1_grid_lbfgs():
    from oracle.precond import Kernel
    N, H, stride = 256, 50, 8
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    osteps = evenly_spaced(H, 5)
    truth = O.init_field(N, [0], kind=0, k0=10.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(stride, osteps))
    fg = O.first_guess(N, stride, mo[0])
    kern = Kernel(1, 0.05, 0)
    out = {"obs_steps": np.array(osteps), "obs": np.asarray(mo), "first_guess": fg}
    for k in (1, 5, 10):
        w, hist, it, status = O.assimilate(fg, ph, H, Obs(stride, osteps, mo), kern, "lbfgs", k, 10)
        assert status == 0 and it == k, (status, it)
        out[f"omega_{k}"] = w
        out[f"J_hist_{k}"] = np.array(hist)
        print(f"c1 grid L-BFGS: {k} iterations, J {hist[0]:.6e} -> {hist[-1]:.6e}", flush=True)
    np.savez(os.path.join(HERE, "c1_grid_lbfgs.npz"), **out)


def c2_grid_lbfgs():
    from oracle.precond import Kernel
    N, H, stride, every = 512, 40, 16, 2
    ph = Physics(N=N, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    osteps = [0, 20, 40]
    truth = O.init_field(N, [1], kind=0, k0=6.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(stride, osteps))
    fg = O.first_guess(N, stride, mo[0])
    kern = Kernel(2, 0.5, 0)
    out = {"obs_steps": np.array(osteps), "obs": np.asarray(mo), "first_guess": fg, "sample_every": np.array(every)}
    for k in (1, 3, 5):
        w, hist, it, status = O.assimilate(fg, ph, H, Obs(stride, osteps, mo), kern, "lbfgs", k, 10)
        assert status == 0 and it == k, (status, it)
        out[f"omega_{k}"] = np.asarray(w)[::every, ::every].copy()
        out[f"J_hist_{k}"] = np.array(hist)
        print(f"c2 grid L-BFGS: {k} iterations, J {hist[0]:.6e} -> {hist[-1]:.6e}", flush=True)
    np.savez(os.path.join(HERE, "c2_grid_lbfgs.npz"), **out)


def grid1024_50_steps():
    N, H, stride, every = 1024, 50, 16, 4
    ph = Physics(N=N, nu=1e-4, dt=5e-4)
    osteps = [0, 25, 50]
    w0 = O.init_field(N, [3], kind=0, k0=N / 25.0, target=0.5)[0]
    truth = O.init_field(N, [4], kind=0, k0=N / 25.0, target=0.5)[0]
    omega_T = O.forward(w0, ph, H)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(stride, osteps))
    J, g = O.adjoint_gradient(w0, ph, H, Obs(stride, osteps, mo))
    np.savez(os.path.join(HERE, "grid1024_50_steps.npz"), obs_steps=np.array(osteps), obs=np.asarray(mo),
             sample_every=np.array(every), omega_T=np.asarray(omega_T)[::every, ::every].copy(), J=np.array(J),
             grad=np.asarray(g)[::every, ::every].copy())


if __name__ == "__main__":
    which = sys.argv[1:] or ["c1", "ensemble", "c2", "lbfgs", "c2lbfgs", "1024"]
    if "c1" in which:
        c1_full_horizon()
    if "ensemble" in which:
        ensemble_member17()
    if "c2" in which:
        c2_100_steps()
    if "lbfgs" in which:
        c1_grid_lbfgs()
    if "c2lbfgs" in which:
        c2_grid_lbfgs()
    if "1024" in which:
        grid1024_50_steps()
