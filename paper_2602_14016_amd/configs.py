"""Named workloads of the hot path and a runner.

    python -m paper_2602_14016_amd.configs c0|c1|c2|c3|sweep|controls|longwindow [--iters K] [--horizon H]

c0  decaying turbulence, 64^2, nu = 1e-3, Gaussian random field (k0 = 4,
    energy 0.5), 200 RK4 steps at dt = 5e-3, velocity at every 4th grid point
    at the final time, first guess 0, 5 steepest-descent steps with
    W = exp(-0.1 |k|).
c1  decaying turbulence, 256^2, nu = 1e-4, random phases (k0 = 10), 1000
    steps at dt = 2e-3, velocity at 8 x 8-stride probes at 5 evenly spaced
    times, interpolated first guess, 50 L-BFGS iterations for each of W = 1,
    exp(-0.05 |k|), |k|^-1; checkpoints every 50 steps.
c2  forced Kolmogorov flow, 512^2, nu = 1/40, drag 0.1, f_x = sin 4y, spin-up
    of 5000 steps from noise of RMS 1e-2, horizon 2000 at dt = 1e-3,
    observations at 16 x 16 stride every 50 steps, W = |k|^(-2 beta) for beta
    in {0.25, 0.5, 1.0}, 30 L-BFGS iterations.
c3  ensemble of 64 realizations of the c1 spectrum (seeds 0..63), 500
    forward + 500 adjoint steps from a unit u-impulse, shell energies and
    growth rates for |k| = 1..85; with --members M > 64 the ensemble
    statistics of M realizations in batches.  --flow kolmogorov: the paper's
    Kolmogorov flow (512^2, Re = 400, no drag, 40-unit precursor per
    realization) with 150 realizations over T = 8 in batches of 50 (App. C).
sweep  the c1 problem assimilated under 14 preconditioners at once (fractional
    |k|^(-2 alpha), alpha = -2..2, and heat exp(-nu beta |k|^2), beta = -0.1..0.8)
    as one batched solve, timed against one solve per kernel.
controls  the c1 problem with the control variables of Sec. III.A: velocity,
    vorticity and streamfunction (one batched solve) and velocity with the
    Sobolev-regularised cost (lambda = 1e-3).
longwindow  the c1 flow over 20000 steps (64 members) with a 16 GiB workspace,
    below what one checkpoint per segment needs: binomial checkpointing,
    timed and compared bit for bit with the unbudgeted gradient.

Truth fields are seeded synthetic spectra (the paper's truth realizations are
not available); observations are the model's own (twin experiment).
"""

import argparse
import json
import sys
import time
from dataclasses import dataclass, field
from typing import List, Tuple

import torch

from .solver import KernelSpec, Observations, Solver


def evenly_spaced(n_steps, n):
    return sorted({int(round(i * n_steps / (n - 1))) for i in range(n)})


@dataclass
class Config:
    name: str
    N: int
    nu: float
    dt: float
    n_steps: int
    stride: int
    obs_steps: List[int]
    kernels: List[KernelSpec]
    method: str = "lbfgs"
    iters: int = 50
    mu: float = 0.0
    forcing_amp: float = 0.0
    forcing_k: int = 4
    truth_kind: int = 0
    truth_k0: float = 10.0
    truth_target: float = 0.5
    truth_seed: int = 0
    spinup: int = 0
    first_guess: str = "interp"
    ckpt_every: int = 50
    lbfgs_m: int = 10

    def physics(self):
        return dict(nu=self.nu, dt=self.dt, mu=self.mu, forcing_amp=self.forcing_amp, forcing_k=self.forcing_k)


def c0():
    return Config("c0", 64, 1e-3, 5e-3, 200, 4, [200], [KernelSpec(1, 0.1)], method="sd", iters=5,
                  truth_kind=1, truth_k0=4.0, first_guess="zero")


def c1():
    return Config("c1", 256, 1e-4, 2e-3, 1000, 8, evenly_spaced(1000, 5),
                  [KernelSpec(0, 0.0), KernelSpec(1, 0.05), KernelSpec(2, 0.5)], iters=50, truth_k0=10.0)


def c2():
    return Config("c2", 512, 1.0 / 40, 1e-3, 2000, 16, list(range(0, 2001, 50)),
                  [KernelSpec(2, 0.25), KernelSpec(2, 0.5), KernelSpec(2, 1.0)], iters=30, mu=0.1,
                  forcing_amp=1.0, forcing_k=4, truth_kind=2, truth_target=1e-2, spinup=5000)


CONFIGS = {"c0": c0, "c1": c1, "c2": c2}


def sweep_kernels(nu=1e-4, alphas=(-2.0, -1.5, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5, 2.0),
                  betas=(-0.1, 0.1, 0.3, 0.5, 0.8)):
    """Fractional kernels |k|^(-2 alpha) and heat kernels exp(-nu beta |k|^2) (Sec. III.B-C)."""
    return [KernelSpec(2, a) for a in alphas] + [KernelSpec(3, nu * b) for b in betas]


def run_controls(cfg: Config, iters, sobolev=1e-3, verbose=True):
    """The control-variable comparison of Sec. III.A on cfg: velocity, vorticity and
    streamfunction controls (identity kernel, three metrics) as one batched solve, and
    the velocity control with the Sobolev term lambda/2 int |grad u0|^2 of the cost."""
    from .solver import STREAMFUNCTION, VELOCITY, VORTICITY
    s1 = Solver(cfg.N, 1, **cfg.physics())
    truth, obs_vals = truth_and_obs(cfg, s1)
    fg = s1.first_guess(cfg.stride, obs_vals[:, 0].contiguous())
    names = ["u0", "omega0", "psi0"]
    kernels = [KernelSpec(0, 0.0, VELOCITY), KernelSpec(0, 0.0, VORTICITY), KernelSpec(0, 0.0, STREAMFUNCTION)]
    sb = Solver(cfg.N, 3, **cfg.physics())
    obs_b = Observations(cfg.stride, cfg.obs_steps, obs_vals.expand(3, -1, -1, -1, -1).contiguous())
    w, H, it = sb.assimilate(fg.expand(3, -1, -1).contiguous(), cfg.n_steps, obs_b, kernels, "lbfgs", iters,
                             cfg.lbfgs_m, cfg.ckpt_every)
    s1.set_sobolev(sobolev)
    wr, Hr, itr = s1.assimilate(fg, cfg.n_steps, Observations(cfg.stride, cfg.obs_steps, obs_vals), kernels[0],
                                "lbfgs", iters, cfg.lbfgs_m, cfg.ckpt_every)
    ws = torch.cat([w, wr])
    err = (torch.linalg.norm((ws - truth).reshape(4, -1), dim=1) / torch.linalg.norm(truth)).cpu().tolist()
    out = {"config": cfg.name + "-controls", "controls": names + [f"u0+sobolev({sobolev:g})"],
           "iterations": it + itr, "J_history": H + Hr, "rel_err_omega0": err}
    if verbose:
        print(json.dumps(out), flush=True)
    return out


def run_kolmogorov_ensemble(members=150, batch=50, n_steps=8000, spinup=40000, verbose=True):
    """Ensemble adjoint statistics of the forced Kolmogorov flow (App. C) with
    the paper's setup of that flow (Sec. III.E, Table 1): 512^2, Re = 400
    (nu = 1/400), no drag, f_x = sin 4y, dt = 1e-3; each realization is a
    random-phase field (k0 = 4, energy 0.5; seeds 0..members-1) advanced
    `spinup` steps (the 40-time-unit precursor), then a unit u-impulse at the
    centre after n_steps (T = 8) is propagated back; shell energies for |k| =
    1..170, statistics at subset sizes 50, 100, 150."""
    from . import ensemble
    from .autotune import autotune
    N, nu, dt, amp, kf = 512, 1.0 / 400, 1e-3, 1.0, 4
    probe = Solver(N, batch, nu=nu, dt=dt, forcing_amp=amp, forcing_k=kf)
    tiles = {k: v for k, v in autotune(probe, n_steps=8).items() if k in probe.get_tiles()}
    probe.close()
    del probe
    st = ensemble.statistics(N=N, members=members, batch=batch, n_steps=n_steps, nu=nu, dt=dt, k0=4.0,
                             subsets=(50, 100, 150), tiles=tiles, verbose=verbose, forcing_amp=amp, forcing_k=kf,
                             init_kind=0, init_target=0.5, spinup=spinup)
    every = max(1, n_steps // 16)
    out = {"config": "c3-kolmogorov", "members": st.members, "seconds": st.seconds,
           "tau": [float(x) for x in st.tau[::every].cpu()],
           "total_mean": [float(x) for x in st.total_mean[::every].cpu()],
           "total_of_mean": [float(x) for x in st.total_of_mean[::every].cpu()],
           "snr": [float(x) for x in st.snr[::every].cpu()],
           "subsets": {str(n): {"total_mean_at_T": float(v["total_mean"][-1].cpu()),
                                "snr_at_T": float(v["snr"][-1].cpu())} for n, v in st.subsets.items()},
           "mean_energy_shells_at": {f"{float(st.tau[r]):.1f}": [float(x) for x in st.mean_energy[r, :40].cpu()]
                                     for r in (0, n_steps // 4, n_steps // 2, n_steps)}}
    if verbose:
        print(json.dumps(out), flush=True)
    return out


def run_longwindow(N=256, B=64, n_steps=20000, budget_gib=16.0, n_obs=5, stride=8, verbose=True):
    """A long assimilation window under a memory budget (binomial checkpointing).

    The c1 flow (N^2, nu = 1e-4, dt = 2e-3) over n_steps steps, B members,
    observations at n_obs evenly spaced times.  The budget is set below what
    one checkpoint per segment boundary needs at any segment length, so the
    gradient runs with the binomial schedule that fit_checkpointing picks;
    it is timed, then the same gradient without a budget (one checkpoint per
    boundary, longest segments that fit the device), and the two are
    compared bit for bit."""
    from .autotune import autotune
    s = Solver(N, B, nu=1e-4, dt=2e-3)
    tiles = {k: v for k, v in autotune(s, n_steps=8).items() if k in s.get_tiles()}
    s.set_tiles(**tiles)
    steps = evenly_spaced(n_steps, n_obs)
    truth = s.init_field([1000 + b for b in range(B)], kind=0, k0=10.0, target=0.5)
    obs = Observations(stride, steps, s.forward(truth, n_steps, Observations(stride, steps), want_obs=True)["obs"])
    del truth
    w0 = s.init_field(list(range(B)), kind=0, k0=10.0, target=0.5)
    budget = int(budget_gib * (1 << 30))
    s.set_checkpoint_slots(0)
    uniform_floor = min(s.workspace_bytes(n_steps, -(-n_steps // L), len(steps), 0) for L in range(1, n_steps + 1))
    K, slots, fwd = s.fit_checkpointing(n_steps, len(steps), 0, budget_bytes=budget)
    if not K:
        raise SystemExit(f"nothing fits in {budget_gib} GiB")

    def timed_gradient(K_):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J, g = s.adjoint_gradient(w0, n_steps, obs, ckpt_every=K_)
        torch.cuda.synchronize()
        return J, g, time.perf_counter() - t0

    s.set_checkpoint_slots(slots)
    ws_bin = s.workspace_bytes(n_steps, K, len(steps), 0)
    Jb, gb, tb = timed_gradient(K)
    Jb, gb = Jb.cpu(), gb.cpu()
    s._ws = None
    torch.cuda.empty_cache()
    s.set_checkpoint_slots(0)
    Ku = s.fit_ckpt_every(n_steps, len(steps))
    Lu = -(-n_steps // Ku)
    ws_uni = s.workspace_bytes(n_steps, Ku, len(steps), 0)
    Ju, gu, tu = timed_gradient(Ku)
    same = bool(torch.equal(Jb, Ju.cpu()) and torch.equal(gb, gu.cpu()))
    out = {"config": f"longwindow-{N}x{B}-H{n_steps}", "budget_gib": budget_gib,
           "uniform_min_workspace_gib": uniform_floor / (1 << 30),
           "binomial": {"segment_steps": K, "segments": -(-n_steps // K), "slots": slots,
                        "workspace_gib": ws_bin / (1 << 30), "forward_steps": fwd, "seconds": tb},
           "unbudgeted": {"segment_steps": Ku, "segments": Lu, "workspace_gib": ws_uni / (1 << 30),
                          "forward_steps": n_steps + (Lu - 1) * Ku, "seconds": tu},
           "bitwise_equal": same, "grad_finite": bool(torch.isfinite(gb).all())}
    if verbose:
        print(json.dumps(out), flush=True)
    return out


def run_sweep(cfg: Config, kernels, iters, sequential=True, verbose=True):
    """Assimilate cfg once per kernel: all kernels as one batched solve, then (if
    sequential) one solve per kernel; returns timings and per-kernel results."""
    B = len(kernels)
    s1 = Solver(cfg.N, 1, **cfg.physics())
    truth, obs_vals = truth_and_obs(cfg, s1)
    fg = s1.first_guess(cfg.stride, obs_vals[:, 0].contiguous())
    sb = Solver(cfg.N, B, **cfg.physics())
    obs_b = Observations(cfg.stride, cfg.obs_steps, obs_vals.expand(B, -1, -1, -1, -1).contiguous())
    fg_b = fg.expand(B, -1, -1).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w, H, it = sb.assimilate(fg_b, cfg.n_steps, obs_b, kernels, "lbfgs", iters, cfg.lbfgs_m, cfg.ckpt_every)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    err = (torch.linalg.norm((w - truth).reshape(B, -1), dim=1) / torch.linalg.norm(truth)).cpu().tolist()
    out = {"config": cfg.name + "-sweep", "kernels": [[k.kind, k.param] for k in kernels], "iterations": it,
           "J_final": [h[it_b] if it_b >= 0 else None for h, it_b in zip(H, it)], "rel_err_omega0": err,
           "batched_seconds": t_batched}
    if sequential:
        obs1 = Observations(cfg.stride, cfg.obs_steps, obs_vals)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in kernels:
            s1.assimilate(fg, cfg.n_steps, obs1, k, "lbfgs", iters, cfg.lbfgs_m, cfg.ckpt_every)
        torch.cuda.synchronize()
        out["sequential_seconds"] = time.perf_counter() - t0
        out["speedup"] = out["sequential_seconds"] / t_batched
    if verbose:
        print(json.dumps(out), flush=True)
    return out


def velocity_error_in_time(solver: Solver, truth, est, n_steps, n_points=11):
    """The reconstruction error over the window, eps(t) / u_rms (Sec. III.C-D): the RMS velocity
    error of the trajectory started from est against the truth's, over the truth's RMS velocity,
    at n_points evenly spaced steps; velocities on the full grid are stride-1 observations.
    truth is [1, N, N], est [B, N, N]; returns (steps, [B][n_points])."""
    steps = evenly_spaced(n_steps, n_points)
    full = Observations(1, steps)
    B = est.shape[0]
    if solver.B != B:
        raise ValueError("est must have the solver's batch")
    ut = solver.forward(truth.expand(B, -1, -1).contiguous(), n_steps, full, want_obs=True)["obs"]
    ue = solver.forward(est, n_steps, full, want_obs=True)["obs"]
    err = ((ue - ut) ** 2).sum(dim=(2, 3, 4)).sqrt() / (ut ** 2).sum(dim=(2, 3, 4)).sqrt()
    return steps, err.cpu().tolist()


def truth_and_obs(cfg: Config, solver: Solver):
    """Seeded truth (after spin-up) and its model observations [B, n_times, 2, M, M]."""
    w = solver.init_field([cfg.truth_seed + b for b in range(solver.B)], kind=cfg.truth_kind, k0=cfg.truth_k0,
                          target=cfg.truth_target)
    if cfg.spinup:
        w = solver.forward(w, cfg.spinup)["omega_T"]
    obs = solver.forward(w, cfg.n_steps, Observations(cfg.stride, cfg.obs_steps), want_obs=True)["obs"]
    return w, obs


def run_config(cfg: Config, iters=None, verbose=True, batched=False):
    """Run the assimilation of cfg once per kernel (with batched, all kernels as one
    solve, one member per kernel); returns a list of result dicts."""
    if batched:
        return _run_config_batched(cfg, iters, verbose)
    s = Solver(cfg.N, 1, **cfg.physics())
    t0 = time.perf_counter()
    truth, obs_vals = truth_and_obs(cfg, s)
    obs = Observations(cfg.stride, cfg.obs_steps, obs_vals)
    if cfg.first_guess == "interp" and cfg.obs_steps[0] == 0:
        fg = s.first_guess(cfg.stride, obs_vals[:, 0].contiguous())
    else:
        fg = torch.zeros_like(truth)
    setup_s = time.perf_counter() - t0
    K = cfg.ckpt_every if cfg.ckpt_every > 0 else s.fit_ckpt_every(cfg.n_steps, len(cfg.obs_steps), cfg.lbfgs_m)
    out = []
    for kern in cfg.kernels:
        t1 = time.perf_counter()
        w, H, it = s.assimilate(fg, cfg.n_steps, obs, kern, cfg.method, iters or cfg.iters, cfg.lbfgs_m, K)
        torch.cuda.synchronize()
        err = float(torch.linalg.norm(w - truth) / torch.linalg.norm(truth))
        secs = time.perf_counter() - t1
        t_steps, eps = velocity_error_in_time(s, truth, w, cfg.n_steps)
        rec = {"config": cfg.name, "kernel": [kern.kind, kern.param, kern.metric], "iterations": it[0],
               "ckpt_every": K, "J": [h for h in H[0] if h == h], "rel_err_omega0": err, "seconds": secs,
               "setup_seconds": setup_s, "eps_over_urms": {"steps": t_steps, "value": eps[0]}}
        out.append(rec)
        if verbose:
            print(json.dumps(rec), flush=True)
    return out


def _run_config_batched(cfg: Config, iters, verbose):
    nk = len(cfg.kernels)
    s1 = Solver(cfg.N, 1, **cfg.physics())
    t0 = time.perf_counter()
    truth, obs_vals = truth_and_obs(cfg, s1)
    if cfg.first_guess == "interp" and cfg.obs_steps[0] == 0:
        fg = s1.first_guess(cfg.stride, obs_vals[:, 0].contiguous())
    else:
        fg = torch.zeros_like(truth)
    setup_s = time.perf_counter() - t0
    s1.close()
    del s1
    s = Solver(cfg.N, nk, **cfg.physics())
    obs = Observations(cfg.stride, cfg.obs_steps, obs_vals.expand(nk, -1, -1, -1, -1).contiguous())
    K = cfg.ckpt_every if cfg.ckpt_every > 0 else s.fit_ckpt_every(cfg.n_steps, len(cfg.obs_steps), cfg.lbfgs_m)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w, H, it = s.assimilate(fg.expand(nk, -1, -1).contiguous(), cfg.n_steps, obs, list(cfg.kernels), cfg.method,
                            iters or cfg.iters, cfg.lbfgs_m, K)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t1
    t_steps, eps = velocity_error_in_time(s, truth, w, cfg.n_steps)
    out = []
    for b, kern in enumerate(cfg.kernels):
        err = float(torch.linalg.norm(w[b] - truth[0]) / torch.linalg.norm(truth[0]))
        rec = {"config": cfg.name + "-batched", "kernel": [kern.kind, kern.param, kern.metric], "iterations": it[b],
               "ckpt_every": K, "J": [h for h in H[b] if h == h], "rel_err_omega0": err, "seconds_all_kernels": secs,
               "setup_seconds": setup_s, "eps_over_urms": {"steps": t_steps, "value": eps[b]}}
        out.append(rec)
        if verbose:
            print(json.dumps(rec), flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("config", choices=sorted(list(CONFIGS) + ["c3", "sweep", "controls", "longwindow"]))
    ap.add_argument("--iters", type=int, default=None)
    ap.add_argument("--horizon", type=int, default=None)
    ap.add_argument("--members", type=int, default=64, help="c3: ensemble size (statistics in batches beyond 64)")
    ap.add_argument("--batch", type=int, default=64, help="c3: members per batched solve")
    ap.add_argument("--budget-gib", type=float, default=16.0, help="longwindow: workspace budget")
    ap.add_argument("--batched", action="store_true", help="c0/c1/c2: all kernels as one batched solve")
    ap.add_argument("--ckpt-every", type=int, default=None,
                    help="c0/c1/c2: checkpoint interval instead of the configuration's (the horizon keeps the "
                         "whole trajectory, 0 the largest that fits in free HBM; results do not depend on it)")
    ap.add_argument("--flow", choices=["hit", "kolmogorov"], default="hit",
                    help="c3: decaying HIT (256^2) or forced Kolmogorov flow (512^2, T = 8; App. C)")
    args = ap.parse_args(argv)
    if args.config == "c3" and args.flow == "kolmogorov":
        run_kolmogorov_ensemble(members=args.members if args.members != 64 else 150,
                                batch=args.batch if args.batch != 64 else 50, n_steps=args.horizon or 8000)
        return
    if args.config == "c3":
        from . import ensemble
        t0 = time.perf_counter()
        H = args.horizon or 500
        res = ensemble.run(n_steps=H, members=min(args.members, args.batch))
        torch.cuda.synchronize()
        out = {"config": "c3", "seconds": time.perf_counter() - t0,
               "growth_rates": [float(x) for x in res.rates.cpu()]}
        if args.members > args.batch:
            from .autotune import autotune
            probe = Solver(256, args.batch, nu=1e-4, dt=2e-3)
            tiles = {k: v for k, v in autotune(probe, n_steps=8).items() if k in probe.get_tiles()}
            probe.close()
            del probe
            st = ensemble.statistics(members=args.members, batch=args.batch, n_steps=H, tiles=tiles, verbose=True)
            every = max(1, H // 20)
            out["statistics"] = {
                "members": st.members, "seconds": st.seconds, "tau": [float(x) for x in st.tau[::every].cpu()],
                "snr": [float(x) for x in st.snr[::every].cpu()],
                "total_mean": [float(x) for x in st.total_mean[::every].cpu()],
                "total_of_mean": [float(x) for x in st.total_of_mean[::every].cpu()],
                "subsets": {str(n): {"snr_at_tau_1": float(v["snr"][min(int(round(1.0 / 2e-3)), H)].cpu())}
                            for n, v in st.subsets.items()}}
        print(json.dumps(out))
        return
    if args.config == "longwindow":
        run_longwindow(B=args.batch, n_steps=args.horizon or 20000, budget_gib=args.budget_gib)
        return
    if args.config == "controls":
        cfg = c1()
        if args.horizon:
            cfg.n_steps = args.horizon
            cfg.obs_steps = evenly_spaced(args.horizon, 5)
        run_controls(cfg, args.iters or 10)
        return
    if args.config == "sweep":
        cfg = c1()
        if args.horizon:
            cfg.n_steps = args.horizon
            cfg.obs_steps = evenly_spaced(args.horizon, 5)
        run_sweep(cfg, sweep_kernels(cfg.nu), args.iters or 10)
        return
    cfg = CONFIGS[args.config]()
    if args.horizon:
        cfg.n_steps = args.horizon
        cfg.obs_steps = [s for s in cfg.obs_steps if s <= args.horizon] or [args.horizon]
    if args.ckpt_every is not None:
        cfg.ckpt_every = args.ckpt_every
    run_config(cfg, args.iters, batched=args.batched)


if __name__ == "__main__":
    main()
