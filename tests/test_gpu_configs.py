"""GPU checks at the configurations' own sizes.

c0 runs in full against the oracle; c1 and c2 are checked against the oracle
at a shortened horizon on their full grids, and c1 in full (256^2, 1000
steps) by central finite differences of the GPU's own cost on 20 directions.
"""

import numpy as np
import pytest
import torch

import oracle as O
import synth
from oracle.model import Obs, Physics
from oracle.precond import Kernel

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def test_c0_full_parity():
    from paper_2602_14016_amd import KernelSpec, Observations, Solver
    print("CASE c0", flush=True)
    N, H = 64, 200
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    truth = O.init_field(N, [0], kind=1, k0=4.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(4, [H]))
    fg = np.zeros((N, N))
    w_ref, h_ref, it_ref, st_ref = O.assimilate(fg, ph, H, Obs(4, [H], mo), Kernel(1, 0.1, 0), "sd", 5)
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    w, Hh, it = s.assimilate(dev(fg[None]), H, Observations(4, [H], dev(mo[None])), KernelSpec(1, 0.1), "sd", 5,
                             ckpt_every=50)
    torch.cuda.synchronize()
    assert it[0] == it_ref == 5
    assert np.allclose(Hh[0], h_ref, rtol=1e-9, atol=0)
    assert rel(w.cpu().numpy()[0], w_ref) < 1e-9
    assert h_ref[-1] < h_ref[0]


def test_c1_shortened_horizon_gradient_parity():
    from paper_2602_14016_amd import Observations, Solver
    print("CASE c1-100", flush=True)
    N, H = 256, 100
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    osteps = synth.evenly_spaced_steps(H, 5)
    truth = O.init_field(N, [0], kind=0, k0=10.0)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(8, osteps))
    w0 = O.init_field(N, [1], kind=0, k0=10.0)[0]
    J_ref, g_ref = O.adjoint_gradient(w0, ph, H, Obs(8, osteps, mo))
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    J, g = s.adjoint_gradient(dev(w0[None]), H, Observations(8, osteps, dev(mo[None])), ckpt_every=50)
    torch.cuda.synchronize()
    assert abs(float(J.cpu()[0]) - J_ref) <= 1e-11 * J_ref
    assert rel(g.cpu().numpy()[0], g_ref) < 1e-9


def _golden(name):
    import os
    return np.load(os.path.join(os.path.dirname(__file__), "golden", name))


def test_c1_full_horizon_gradient_against_oracle():
    """c1 at its full horizon (256^2, nu = 1e-4, 1000 steps at dt = 2e-3, 5
    observation times at stride 8, checkpoints every 50): cost and gradient
    against the oracle's, written by tests/golden/make_oracle_fixtures.py."""
    from paper_2602_14016_amd import Observations, Solver
    print("CASE c1-1000", flush=True)
    N, H = 256, 1000
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    osteps = synth.evenly_spaced_steps(H, 5)
    ref = _golden("c1_full_horizon.npz")
    assert list(ref["obs_steps"]) == list(osteps)
    mo, J_ref, g_ref = ref["obs"], float(ref["J"]), ref["grad"]
    w0 = O.init_field(N, [1], kind=0, k0=10.0, target=0.5)[0]
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    J, g = s.adjoint_gradient(dev(w0[None]), H, Observations(8, osteps, dev(mo[None])), ckpt_every=50)
    torch.cuda.synchronize()
    ej = abs(float(J.cpu()[0]) - J_ref) / J_ref
    eg = rel(g.cpu().numpy()[0], g_ref)
    print("CASE c1-1000 rel J", ej, "rel grad", eg, flush=True)
    assert ej <= 1e-11
    assert eg < 1e-9
    # the same gradient through the autograd path as the configuration runs it: checkpoints
    # every 50 steps in the forward, segment recomputation in the backward, grad_output 1
    from paper_2602_14016_amd.autograd import adjoint_cost
    print("CASE c1-1000 autograd", flush=True)
    w = dev(w0[None]).requires_grad_(True)
    Ja = adjoint_cost(w, s, H, Observations(8, osteps, dev(mo[None])), 50)
    Ja.sum().backward()
    ea = rel(w.grad.detach().cpu().numpy()[0], g_ref)
    print("CASE c1-1000 autograd rel J", abs(float(Ja.detach().cpu()[0]) - J_ref) / J_ref, "rel grad", ea, flush=True)
    assert abs(float(Ja.detach().cpu()[0]) - J_ref) <= 1e-11 * J_ref
    assert ea < 1e-9


def test_c1_full_finite_differences():
    """The differentiation configuration as specified: the gradient from the autograd path
    (checkpoints every 50 steps, segment recomputation in the backward) against central finite
    differences (eps = 1e-6) of the cost on 20 random directions."""
    from paper_2602_14016_amd import Observations, Solver
    from paper_2602_14016_amd.autograd import adjoint_cost
    print("CASE c1-fd", flush=True)
    N, H, ndir = 256, 1000, 20
    s1 = Solver(N, 1, nu=1e-4, dt=2e-3)
    osteps = synth.evenly_spaced_steps(H, 5)
    truth = s1.init_field([0], kind=0, k0=10.0)
    mo = s1.forward(truth, H, Observations(8, osteps), want_obs=True)["obs"]
    fg = s1.first_guess(8, mo[:, 0].contiguous())
    obs1 = Observations(8, osteps, mo)
    w = fg.clone().requires_grad_(True)
    adjoint_cost(w, s1, H, obs1, 50).sum().backward()
    g = w.grad.detach()
    rms = float(fg.pow(2).mean().sqrt())
    d = torch.stack([torch.from_numpy(synth.normal_field((N, N), 1000 + i)) for i in range(ndir)]).cuda()
    d = d * (rms / d.pow(2).mean(dim=(1, 2), keepdim=True).sqrt())
    sB = Solver(N, ndir, nu=1e-4, dt=2e-3)
    obsB = Observations(8, osteps, mo.expand(ndir, -1, -1, -1, -1).contiguous())
    eps = 1e-6
    Jp = sB.forward((fg + eps * d).contiguous(), H, obsB)["J"]
    Jm = sB.forward((fg - eps * d).contiguous(), H, obsB)["J"]
    fd = ((Jp - Jm) / (2 * eps)).cpu().numpy()
    ad = (g * d).sum(dim=(1, 2)).cpu().numpy()
    relerr = np.abs(fd - ad) / np.abs(ad)
    print("c1 FD relative errors: max %.2e median %.2e" % (relerr.max(), np.median(relerr)), flush=True)
    assert np.all(relerr < 1e-6), relerr


def test_c2_grid_short_parity():
    from paper_2602_14016_amd import Observations, Solver
    print("CASE c2-512", flush=True)
    N, H = 512, 3
    ph = Physics(N=N, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    w0 = O.init_field(N, [0], kind=0, k0=6.0, target=0.5)[0]
    truth = O.init_field(N, [1], kind=0, k0=6.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(16, [0, H]))
    J_ref, g_ref = O.adjoint_gradient(w0, ph, H, Obs(16, [0, H], mo))
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt, mu=ph.mu, forcing_amp=1.0, forcing_k=4)
    J, g = s.adjoint_gradient(dev(w0[None]), H, Observations(16, [0, H], dev(mo[None])), ckpt_every=2)
    torch.cuda.synchronize()
    assert abs(float(J.cpu()[0]) - J_ref) <= 1e-11 * J_ref
    assert rel(g.cpu().numpy()[0], g_ref) < 1e-9


def test_c2_100_step_field_and_gradient_against_oracle():
    """The Kolmogorov configuration's physics on its 512^2 grid over 100 steps (forcing, drag,
    nu = 1/40, dt = 1e-3): the field after 100 steps within 1e-11 and the cost and gradient of a
    3-time observation window (stride 16) within 1e-11 and 1e-9 of the oracle's, stored by
    tests/golden/make_oracle_fixtures.py."""
    from paper_2602_14016_amd import Observations, Solver
    print("CASE c2-100", flush=True)
    N, H = 512, 100
    ref = _golden("c2_100_steps.npz")
    w0 = O.init_field(N, [0], kind=0, k0=6.0, target=0.5)[0]
    s = Solver(N, 1, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    wT = s.forward(dev(w0[None]), H)["omega_T"]
    osteps = [int(x) for x in ref["obs_steps"]]
    J, g = s.adjoint_gradient(dev(w0[None]), H, Observations(16, osteps, dev(ref["obs"][None])), ckpt_every=25)
    torch.cuda.synchronize()
    assert rel(wT.cpu().numpy()[0], ref["omega_T"]) < 1e-11
    assert abs(float(J.cpu()[0]) - float(ref["J"])) <= 1e-11 * float(ref["J"])
    assert rel(g.cpu().numpy()[0], ref["grad"]) < 1e-9


def test_c1_grid_lbfgs_iterates_against_oracle():
    """L-BFGS at the differentiation configuration's grid and physics (256^2, nu = 1e-4, dt =
    2e-3) over a 50-step window (5 observation times, stride 8), kernel exp(-0.05|k|), memory 10,
    from the oracle's interpolated first guess: the cost after each of 10 iterations and the
    estimates after 1, 5 and 10 iterations against the oracle's (1e-9), stored by
    tests/golden/make_oracle_fixtures.py; and the library's own first guess from the t = 0 probes
    against the oracle's."""
    from paper_2602_14016_amd import KernelSpec, Observations, Solver
    print("CASE c1-grid-lbfgs", flush=True)
    N, H = 256, 50
    ref = _golden("c1_grid_lbfgs.npz")
    osteps = [int(x) for x in ref["obs_steps"]]
    assert osteps == synth.evenly_spaced_steps(H, 5)
    mo = dev(ref["obs"][None])
    s = Solver(N, 1, nu=1e-4, dt=2e-3)
    fg = s.first_guess(8, mo[:, 0].contiguous())
    assert rel(fg.cpu().numpy()[0], ref["first_guess"]) < 1e-13
    obs = Observations(8, osteps, mo)
    for k in (1, 5, 10):
        w, Hh, it = s.assimilate(dev(ref["first_guess"][None]), H, obs, KernelSpec(1, 0.05), "lbfgs", max_iter=k,
                                 lbfgs_m=10, ckpt_every=25)
        href = ref[f"J_hist_{k}"]
        ew = rel(w.cpu().numpy()[0], ref[f"omega_{k}"])
        eh = float(np.max(np.abs(np.array(Hh[0]) - href) / href))
        print(f"CASE c1-grid-lbfgs {k} iterations: rel omega {ew:.2e}, rel J history {eh:.2e}", flush=True)
        assert it[0] == k and len(Hh[0]) == len(href) == k + 1
        assert eh < 1e-9
        assert ew < 1e-9


def test_c2_grid_lbfgs_iterates_against_oracle():
    """L-BFGS at the Kolmogorov configuration's grid and physics (512^2, nu = 1/40, drag 0.1,
    f_x = sin 4y, dt = 1e-3) over a 40-step window (3 observation times, stride 16), kernel
    |k|^-1, memory 10, from the oracle's interpolated first guess: the cost after each of 5
    iterations and the estimates after 1, 3 and 5 (at every 2nd grid point) against the oracle's
    (1e-9), stored by
    tests/golden/make_oracle_fixtures.py; the gradients recompute segments of 20 steps."""
    from paper_2602_14016_amd import KernelSpec, Observations, Solver
    print("CASE c2-grid-lbfgs", flush=True)
    N, H = 512, 40
    ref = _golden("c2_grid_lbfgs.npz")
    osteps = [int(x) for x in ref["obs_steps"]]
    mo = dev(ref["obs"][None])
    s = Solver(N, 1, nu=1.0 / 40, dt=1e-3, mu=0.1, forcing_amp=1.0, forcing_k=4)
    fg = s.first_guess(16, mo[:, 0].contiguous())
    assert rel(fg.cpu().numpy()[0], ref["first_guess"]) < 1e-13
    obs = Observations(16, osteps, mo)
    for k in (1, 3, 5):
        w, Hh, it = s.assimilate(dev(ref["first_guess"][None]), H, obs, KernelSpec(2, 0.5), "lbfgs", max_iter=k,
                                 lbfgs_m=10, ckpt_every=20)
        href = ref[f"J_hist_{k}"]
        ev = int(ref["sample_every"])
        ew = rel(w.cpu().numpy()[0][::ev, ::ev], ref[f"omega_{k}"])
        eh = float(np.max(np.abs(np.array(Hh[0]) - href) / href))
        print(f"CASE c2-grid-lbfgs {k} iterations: rel omega {ew:.2e}, rel J history {eh:.2e}", flush=True)
        assert it[0] == k and len(Hh[0]) == len(href) == k + 1
        assert eh < 1e-9
        assert ew < 1e-9


def test_largest_grid_50_steps_against_oracle():
    """The largest grid (1024^2, nu = 1e-4, dt = 5e-4) over 50 steps: the field after 50 steps
    (1e-11) and the cost (1e-11) and gradient (1e-9) of a 3-time window at stride 16 against the
    oracle's, stored at every 4th grid point in each direction by
    tests/golden/make_oracle_fixtures.py; the gradient recomputes segments of 10 steps.  Checked
    with the default tiles, with the two-wavefront transform plans (variants 1 and 2, whose
    adjoint rows read their twiddles from LDS) and shared column outputs, and with column blocks
    whose LDS exceeds 64 KiB."""
    from paper_2602_14016_amd import Observations, Solver
    print("CASE grid-1024-50", flush=True)
    N, H = 1024, 50
    ref = _golden("grid1024_50_steps.npz")
    ev = int(ref["sample_every"])
    w0 = O.init_field(N, [3], kind=0, k0=N / 25.0, target=0.5)[0]
    s = Solver(N, 1, nu=1e-4, dt=5e-4)
    wT = s.forward(dev(w0[None]), H)["omega_T"].cpu().numpy()[0]
    ef = rel(wT[::ev, ::ev], ref["omega_T"])
    osteps = [int(x) for x in ref["obs_steps"]]
    assert ef < 1e-11
    for tiles in ({}, dict(row_variant=1, row_teams=2, adj_variant=1, adj_teams=2, col_variant=1, col_block=2,
                           col_split=4),
                  dict(row_variant=2, row_teams=1, adj_variant=2, adj_teams=1, col_variant=2, col_block=1,
                       col_split=2),
                  dict(col_variant=1, col_block=4, col_split=2),     # 84 KiB of LDS per workgroup
                  dict(col_variant=0, col_block=8, col_split=4)):    # 152 KiB
        s.set_tiles(**tiles)
        J, g = s.adjoint_gradient(dev(w0[None]), H, Observations(16, osteps, dev(ref["obs"][None])), ckpt_every=10)
        ej = abs(float(J.cpu()[0]) - float(ref["J"])) / float(ref["J"])
        eg = rel(g.cpu().numpy()[0][::ev, ::ev], ref["grad"])
        print(f"CASE grid-1024-50 {tiles} rel field {ef:.2e} cost {ej:.2e} gradient {eg:.2e}", flush=True)
        assert ej <= 1e-11, tiles
        assert eg < 1e-9, tiles


def test_largest_grid_gradient_parity():
    """1024^2, the largest grid: cost and gradient over 2 steps (one-step segments,
    so the segment recomputation runs) against the oracle, and the same gradient
    with a one-slot snapshot budget, bit for bit."""
    from paper_2602_14016_amd import Observations, Solver
    print("CASE grid-1024", flush=True)
    N, H = 1024, 2
    ph = Physics(N=N, nu=1e-4, dt=1e-3)
    w0 = O.init_field(N, [3], kind=0, k0=20.0, target=0.5)[0]
    truth = O.init_field(N, [4], kind=0, k0=20.0, target=0.5)[0]
    _, _, mo = O.forward(truth, ph, H, Obs(32, [0, H]))
    J_ref, g_ref = O.adjoint_gradient(w0, ph, H, Obs(32, [0, H], mo))
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    obs = Observations(32, [0, H], dev(mo[None]))
    J, g = s.adjoint_gradient(dev(w0[None]), H, obs, ckpt_every=1)
    J, g = J.cpu().numpy(), g.cpu().numpy()
    assert abs(float(J[0]) - J_ref) <= 1e-11 * J_ref
    assert rel(g[0], g_ref) < 1e-9
    s.set_checkpoint_slots(1)
    Jb, gb = s.adjoint_gradient(dev(w0[None]), H, obs, ckpt_every=1)
    s.set_checkpoint_slots(0)
    assert np.array_equal(Jb.cpu().numpy(), J) and np.array_equal(gb.cpu().numpy(), g)


def test_c1_full_horizon_divergence_curve():
    """GPU vs oracle vorticity over the full 1000-step c1 horizon (256^2, nu = 1e-4): round-off
    differences grow with the flow's chaotic amplification; the curve is printed, the field bar
    (1e-11) is checked at 100 steps and the growth bounded at 1000."""
    from paper_2602_14016_amd import Solver
    print("CASE c1-divergence", flush=True)
    N, H, every = 256, 1000, 100
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    w = O.init_field(N, [0], kind=0, k0=10.0)[0]
    s = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    wg = dev(w[None])
    curve = []
    for n in range(every, H + 1, every):
        w, _, _ = O.forward(w, ph, every, None)
        wg = s.forward(wg, every)["omega_T"]
        curve.append((n, rel(wg.cpu().numpy()[0], w)))
        print("c1 divergence step %4d: %.3e" % curve[-1], flush=True)
    assert curve[0][1] <= 1e-11
    assert curve[-1][1] <= 1e-8


def _impulse_row0(N, n_shells):
    """Shell energies of the terminal adjoint of a unit u-impulse at a grid point:
    lambda_hat = conj(i ky / |k|^2) times a unit-modulus phase on the band, so shell
    k holds sum 1/2 |k|^2 ky^2 / |k|^4 / N^4 over its band modes (any flow, any point)."""
    Kc = (N - 1) // 3
    out = np.zeros(n_shells)
    for ky in range(-Kc, Kc + 1):
        for kx in range(-Kc, Kc + 1):
            k2 = kx * kx + ky * ky
            if k2 == 0:
                continue
            sh = int(np.floor(np.sqrt(k2)))
            while sh * sh > k2:
                sh -= 1
            while (sh + 1) * (sh + 1) <= k2:
                sh += 1
            if 1 <= sh <= n_shells:
                out[sh - 1] += 0.5 * ky * ky / k2
    return out / float(N) ** 4


def test_ensemble_workload_in_its_launch_configuration():
    """The ensemble workload at its full size (64 members of 256^2, nu = 1e-4,
    dt = 2e-3, 500 forward + 500 adjoint steps, impulse at the centre, 85
    shells) with autotuned tiles and the whole trajectory kept, as timed:
    the terminal row against its closed form for every member, two sampled
    members over the whole horizon against one-member solves with default
    tiles and checkpoints every 50 steps, the same configured solver against
    the oracle over a 10-step horizon on two sampled members, and one sampled
    member against the oracle over the whole horizon."""
    from paper_2602_14016_amd import Solver
    from paper_2602_14016_amd.autotune import autotune
    N, B, H, nsh = 256, 64, 500, 85
    ph = Physics(N=N, nu=1e-4, dt=2e-3)
    print("CASE ensemble-workload setup", flush=True)
    w0np = O.init_field(N, list(range(B)), kind=0, k0=10.0, target=0.5)
    w0 = dev(w0np)
    s = Solver(N, B, nu=ph.nu, dt=ph.dt)
    autotune(s, w0, n_steps=8)
    K = s.fit_ckpt_every(H)
    assert K == H, "the whole trajectory should fit on this device"
    print("CASE ensemble-workload full", s.get_tiles(), K, flush=True)
    shells, _ = s.adjoint_impulse(w0, H, N // 2, N // 2, nsh, ckpt_every=K)
    shells = shells.cpu().numpy()
    assert shells.shape == (B, H + 1, nsh) and np.all(np.isfinite(shells))
    row0 = _impulse_row0(N, nsh)
    for b in range(B):
        assert rel(shells[b, 0], row0) < 1e-12
    ref_solver = Solver(N, 1, nu=ph.nu, dt=ph.dt)
    for b in (5, 50):
        print("CASE ensemble-workload member", b, flush=True)
        one, _ = ref_solver.adjoint_impulse(w0[b:b + 1].contiguous(), H, N // 2, N // 2, nsh, ckpt_every=50)
        assert rel(shells[b], one.cpu().numpy()[0]) < 1e-9
    print("CASE ensemble-workload oracle", flush=True)
    short, _ = s.adjoint_impulse(w0, 10, N // 2, N // 2, nsh, ckpt_every=10)
    short = short.cpu().numpy()
    for b in (0, 63):
        ref = O.impulse_adjoint(w0np[b], ph, 10, N // 2, N // 2, nsh)[0]
        assert rel(short[b], ref) < 1e-9
    # one sampled member over the whole 500 + 500-step horizon against the oracle's shells,
    # written by tests/golden/make_oracle_fixtures.py from the same seed
    print("CASE ensemble-workload oracle full horizon, member 17", flush=True)
    ref = _golden("ensemble_member17.npz")["shells"]
    err = rel(shells[17], ref)
    print("CASE ensemble-workload member 17 rel", err, flush=True)
    assert err < 1e-9
