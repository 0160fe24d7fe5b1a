"""GPU: binomial checkpointing changes only the schedule, never the result.

With a snapshot budget smaller than one state per segment boundary the
library reverses the segments by the binomial schedule, re-advancing from
the few states it keeps.  Every forward step it recomputes runs the same
kernels on the same state, so gradients, costs, impulse responses and
assimilation iterates must equal, bit for bit, those of one checkpoint per
boundary; the gradient is also checked against the oracle.
"""

import numpy as np
import pytest
import torch

import oracle as O
from oracle.model import Obs, Physics

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-9


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def announce(*a):
    print("CASE", *a, flush=True)


def _solver(N, B, ph):
    from paper_2602_14016_amd import Solver
    return Solver(N, B=B, nu=ph.nu, dt=ph.dt, mu=ph.mu, forcing_amp=ph.forcing_amp, forcing_k=ph.forcing_k)


def _twin(N, ph, steps, obs_steps, stride, seed):
    truth = O.init_field(N, [seed], kind=0, k0=min(4.0, N / 4))[0]
    return O.forward(truth, ph, steps, Obs(stride, obs_steps))[2]


def test_schedule_beyond_the_segment_cap_is_refused():
    """A binomial schedule is a host list of about two actions per segment, bounded at 2^22
    segments: a longer scheduled solve is refused before anything is enqueued, the uniform
    layout (no snapshot budget) is not affected by the bound, and the context still solves."""
    from paper_2602_14016_amd.native import PaError
    announce("schedule-cap")
    ph = Physics(N=8, nu=1e-2, dt=5e-3)
    s = _solver(8, 1, ph)
    w0 = s.init_field([0], kind=0, k0=2.0)
    s.set_checkpoint_slots(2)
    with pytest.raises(PaError, match="PA_MAX_SCHEDULE_SEGMENTS"):
        s.adjoint_impulse(w0, (1 << 22) + 1, 3, 5, 2, ckpt_every=1)
    sh2 = host(s.adjoint_impulse(w0, 6, 3, 5, 2, ckpt_every=1)[0])
    s.set_checkpoint_slots(0)
    sh0 = host(s.adjoint_impulse(w0, 6, 3, 5, 2, ckpt_every=1)[0])
    assert np.array_equal(sh2, sh0)


def test_binomial_gradient_equals_uniform_bitwise_and_oracle():
    from paper_2602_14016_amd import Observations
    N, B, steps = 32, 2, 37                      # ragged: the last segment is shorter
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    osteps = [0, 9, 20, 37]
    w0 = O.init_field(N, [3, 4], kind=0, k0=4.0)
    mo = np.stack([_twin(N, ph, steps, osteps, 4, seed=30 + b) for b in range(B)])
    s = _solver(N, B, ph)
    obs = Observations(4, osteps, dev(mo))
    for lam in (0.0, 2e-3):
        s.set_sobolev(lam)
        for K in (1, 3, 5):
            L = -(-steps // K)
            s.set_checkpoint_slots(0)
            J0, g0 = s.adjoint_gradient(dev(w0), steps, obs, ckpt_every=K)
            J0, g0 = host(J0), host(g0)
            for slots in sorted({1, 2, 3, 5, L - 1, L} & set(range(1, L + 1))):
                announce("binomial-gradient", f"lam={lam}", f"K={K}", f"L={L}", f"slots={slots}")
                s.set_checkpoint_slots(slots)
                J, g = s.adjoint_gradient(dev(w0), steps, obs, ckpt_every=K)
                assert np.array_equal(host(J), J0), (K, slots)
                assert np.array_equal(host(g), g0), (K, slots)
        s.set_checkpoint_slots(3)
        for b in range(B):
            Jr, gr = O.adjoint_gradient(w0[b], ph, steps, Obs(4, osteps, mo[b]), sobolev=lam)
            assert abs(float(J0[b]) - Jr) <= 1e-11 * Jr
            assert rel(g0[b], gr) < GRAD_TOL
    s.set_sobolev(0.0)
    s.set_checkpoint_slots(0)


def test_binomial_workspace_is_smaller_by_the_dropped_states():
    N, B, steps, K = 64, 3, 120, 4
    s = _solver(N, B, Physics(N=N, nu=1e-3, dt=5e-3))
    L = steps // K
    s.set_checkpoint_slots(0)
    full = s.workspace_bytes(steps, K, 2, 0)
    s.set_checkpoint_slots(4)
    small = s.workspace_bytes(steps, K, 2, 0)
    Kc = (N - 1) // 3
    state = B * (2 * Kc + 1) * (-(-(Kc + 1) // 8) * 8) * 16
    assert abs((full - small) - (L + 1 - 4) * state) <= 512
    s.set_checkpoint_slots(L + 1)      # more slots than boundaries: one per boundary
    assert s.workspace_bytes(steps, K, 2, 0) == full
    s.set_checkpoint_slots(0)


def test_binomial_impulse_response_bitwise():
    N, B, steps = 32, 3, 30
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    s = _solver(N, B, ph)
    w0 = s.init_field([7, 8, 9], kind=0, k0=4.0, target=0.5)
    s.set_checkpoint_slots(0)
    sh0, f0 = s.adjoint_impulse(w0, steps, N // 2, N // 3, 10, ckpt_every=2, want_field=True)
    sh0, f0 = host(sh0), host(f0)
    for slots in (1, 2, 4):
        announce("binomial-impulse", f"slots={slots}")
        s.set_checkpoint_slots(slots)
        sh, f = s.adjoint_impulse(w0, steps, N // 2, N // 3, 10, ckpt_every=2, want_field=True)
        assert np.array_equal(host(sh), sh0)
        assert np.array_equal(host(f), f0)
    s.set_checkpoint_slots(0)


def test_binomial_assimilation_bitwise():
    from paper_2602_14016_amd import KernelSpec, Observations
    N, B, steps = 32, 2, 24
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    osteps = [0, 8, 16, 24]
    mo = np.stack([_twin(N, ph, steps, osteps, 4, seed=40 + b) for b in range(B)])
    s = _solver(N, B, ph)
    obs = Observations(4, osteps, dev(mo))
    fg = dev(O.init_field(N, [50, 51], kind=0, k0=4.0))
    k = KernelSpec(1, 0.1, 1)
    s.set_checkpoint_slots(0)
    w0, H0, it0 = s.assimilate(fg.clone(), steps, obs, k, "lbfgs", 4, 3, ckpt_every=3)
    w0 = host(w0)
    announce("binomial-assimilate")
    s.set_checkpoint_slots(2)
    w, H, it = s.assimilate(fg.clone(), steps, obs, k, "lbfgs", 4, 3, ckpt_every=3)
    assert it == it0
    assert np.array_equal(np.array(H), np.array(H0), equal_nan=True)
    assert np.array_equal(host(w), w0)
    s.set_checkpoint_slots(0)


def test_fit_checkpointing_under_a_tight_budget():
    from paper_2602_14016_amd import Observations
    N, B, steps = 32, 2, 40
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    osteps = [0, 20, 40]
    mo = np.stack([_twin(N, ph, steps, osteps, 4, seed=60 + b) for b in range(B)])
    s = _solver(N, B, ph)
    obs = Observations(4, osteps, dev(mo))
    w0 = dev(O.init_field(N, [61, 62], kind=0, k0=4.0))
    s.set_checkpoint_slots(0)
    J0, g0 = s.adjoint_gradient(w0, steps, obs, ckpt_every=40)
    J0, g0 = host(J0), host(g0)
    # a budget below what one state per boundary needs at any segment length
    s.set_checkpoint_slots(0)
    floor = min(s.workspace_bytes(steps, K, len(osteps), 0) for K in range(1, steps + 1))
    K, slots, fwd = s.fit_checkpointing(steps, len(osteps), 0, budget_bytes=floor - 1)
    announce("fit-checkpointing", K, slots, fwd)
    assert K >= 1 and slots >= 1
    s.set_checkpoint_slots(slots)
    assert s.workspace_bytes(steps, K, len(osteps), 0) + 256 <= floor - 1
    J, g = s.adjoint_gradient(w0, steps, obs, ckpt_every=K)
    assert np.array_equal(host(J), J0)
    assert np.array_equal(host(g), g0)
    s.set_checkpoint_slots(0)


def test_budget_leaves_the_caller_checkpoint_path_unchanged():
    """pa_forward and pa_adjoint_from_checkpoints keep the caller's one-state-per-boundary
    layout under a snapshot budget: the autograd path (which uses them) gives the uniform
    gradient bit for bit, and so does the budgeted pa_adjoint_gradient."""
    from paper_2602_14016_amd import Observations
    from paper_2602_14016_amd.autograd import adjoint_cost
    N, B, steps, K = 32, 2, 26, 3
    ph = Physics(N=N, nu=1e-3, dt=5e-3)
    osteps = [0, 13, 26]
    mo = np.stack([_twin(N, ph, steps, osteps, 4, seed=70 + b) for b in range(B)])
    s = _solver(N, B, ph)
    obs = Observations(4, osteps, dev(mo))
    w0np = O.init_field(N, [71, 72], kind=0, k0=4.0)
    s.set_checkpoint_slots(0)
    J0, g0 = s.adjoint_gradient(dev(w0np), steps, obs, ckpt_every=K)
    J0, g0 = host(J0), host(g0)
    announce("budget-autograd")
    s.set_checkpoint_slots(2)
    w0 = dev(w0np).requires_grad_(True)
    J = adjoint_cost(w0, s, steps, obs, K)
    J.sum().backward()
    assert np.array_equal(host(J.detach()), J0)
    assert np.array_equal(host(w0.grad), g0)
    Jb, gb = s.adjoint_gradient(dev(w0np), steps, obs, ckpt_every=K)
    assert np.array_equal(host(Jb), J0) and np.array_equal(host(gb), g0)
    s.set_checkpoint_slots(0)


def test_graph_capture_of_a_budgeted_solve():
    """A budgeted impulse solve captured in a HIP graph replays the uniform result,
    with eager work between the replays."""
    from paper_2602_14016_amd.graph import CapturedSolve
    N, B, steps, K = 64, 3, 14, 3
    s = _solver(N, B, Physics(N=N, nu=1e-3, dt=5e-3))
    w0 = s.init_field([5, 6, 7], kind=0, k0=4.0, target=0.5)
    s.set_checkpoint_slots(0)
    sh0, f0 = s.adjoint_impulse(w0, steps, 10, 20, 8, ckpt_every=K, want_field=True)
    sh0, f0 = sh0.clone(), f0.clone()
    announce("budget-graph")
    s.set_checkpoint_slots(2)
    cap = CapturedSolve(lambda: s.adjoint_impulse(w0, steps, 10, 20, 8, ckpt_every=K, want_field=True))
    for rep in range(3):
        sh, f = cap.replay()
        torch.cuda.synchronize()
        assert torch.equal(sh, sh0) and torch.equal(f, f0), rep
        s.forward(w0, 3)
        torch.cuda.synchronize()
    s.set_checkpoint_slots(0)
