"""GPU test of the continuous-batching server: requests of one grid and flow
batch across horizons, strides and kernels; every request's result is the same
alone and in a mix and matches the oracle's solve of it; oversize requests are
rejected alone, and latency is recorded."""

import numpy as np
import pytest
import torch

import oracle as O
from oracle.model import Obs, Physics
from oracle.precond import Kernel

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _physics(flow, N):
    from paper_2602_14016_amd.serving import physics_for
    ph = physics_for(flow, N)
    return Physics(N=N, nu=ph["nu"], dt=ph["dt"], mu=ph["mu"], forcing_amp=ph["forcing_amp"],
                   forcing_k=ph["forcing_k"])


def _make_requests(seed=0, specs=None, arrivals=None):
    """Requests whose observations come from oracle truth runs (seeded fields, twin experiment)."""
    from paper_2602_14016_amd import KernelSpec
    from paper_2602_14016_amd.serving import Request, poisson_arrivals
    specs = specs or [(32, "decaying", 40, 4), (64, "kolmogorov", 30, 8), (32, "decaying", 40, 4),
                      (64, "decaying", 24, 4), (32, "kolmogorov", 20, 2), (64, "decaying", 24, 4)]
    kernels = [KernelSpec(0, 0.0), KernelSpec(1, 0.05), KernelSpec(2, 0.5)]
    if arrivals is None:
        arrivals = poisson_arrivals(len(specs), rate=50.0, seed=seed)
    reqs = []
    for i, (N, flow, H, stride) in enumerate(specs):
        truth = O.init_field(N, [100 + i], kind=0 if flow == "decaying" else 2, k0=max(2.0, N / 25),
                             target=0.5 if flow == "decaying" else 1e-2)[0]
        steps = [0, H // 2, H]
        obs = torch.from_numpy(np.ascontiguousarray(O.forward(truth, _physics(flow, N), H, Obs(stride, steps))[2]))
        kern = kernels[i % 3] if i != 3 else kernels[2]
        reqs.append(Request(rid=i, N=N, flow=flow, n_steps=H, stride=stride, obs_steps=steps, obs_values=obs,
                            kernel=kern, iters=3, lbfgs_m=3, ckpt_every=10, arrival=float(arrivals[i])))
    return reqs


def _oracle_solve(r):
    """The oracle's 4D-Var of request r alone: interpolated first guess, L-BFGS."""
    N = r.N
    mo = r.obs_values.numpy()
    fg = O.first_guess(N, r.stride, mo[0])
    k = r.kernel
    return O.assimilate(fg, _physics(r.flow, N), r.n_steps, Obs(r.stride, r.obs_steps, mo),
                        Kernel(k.kind, k.param, k.metric), "lbfgs", r.iters, r.lbfgs_m)


def test_batched_groups_equal_alone_and_oracle():
    """Requests of one grid and flow that wait together run as one batched solve whatever their
    horizons, strides and kernels: each served result is bitwise the same alone and in the batch,
    and matches the oracle's solve of that request (final field and cost history, 1e-9)."""
    from paper_2602_14016_amd.serving import Server, latency_stats
    print("CASE serving-batched", flush=True)
    specs = [(32, "decaying", 40, 4), (32, "decaying", 24, 2), (64, "kolmogorov", 30, 8), (32, "decaying", 16, 8),
             (64, "kolmogorov", 12, 4), (64, "decaying", 20, 4)]
    reqs = _make_requests(specs=specs, arrivals=[0.0] * len(specs))
    mix = Server(hbm_budget_bytes=8 << 30, slots=2, max_batch=8).run_trace(reqs)
    assert all(r.status == "ok" for r in mix.values()), {k: v.status for k, v in mix.items()}
    assert [mix[i].batch for i in range(len(specs))] == [3, 3, 2, 3, 2, 1]
    for r in reqs:
        print("CASE serving-batched request", r.rid, r.N, r.flow, r.n_steps, r.stride, flush=True)
        alone = Server(hbm_budget_bytes=8 << 30, slots=1).run_trace([r])[r.rid]
        assert alone.status == "ok" and alone.batch == 1
        a, m = alone.omega0.numpy(), mix[r.rid].omega0.numpy()
        assert np.array_equal(a, m), (r.rid, float(np.abs(a - m).max()))
        assert alone.J_hist == mix[r.rid].J_hist
        w_ref, h_ref, it_ref, st_ref = _oracle_solve(r)
        assert st_ref == 0 and mix[r.rid].iters == it_ref == r.iters
        assert np.allclose(mix[r.rid].J_hist, h_ref, rtol=1e-9, atol=0), (r.rid, mix[r.rid].J_hist, h_ref)
        assert rel(m, w_ref) < 1e-9, (r.rid, rel(m, w_ref))
    st = latency_stats(mix)
    assert st["n"] == len(reqs) and st["p99_s"] >= st["p50_s"] > 0


def test_alone_equals_mix_and_latency():
    """Poisson arrivals over 3 slots: every request's result is bitwise the same alone and in the
    mix, and matches the oracle's solve of it."""
    from paper_2602_14016_amd.serving import Server, latency_stats
    print("CASE serving", flush=True)
    reqs = _make_requests()
    mix = Server(hbm_budget_bytes=8 << 30, slots=3).run_trace(reqs)
    assert all(r.status == "ok" for r in mix.values()), {k: v.status for k, v in mix.items()}
    for r in reqs:
        alone = Server(hbm_budget_bytes=8 << 30, slots=1).run_trace([r])[r.rid]
        assert alone.status == "ok"
        a, m = alone.omega0.numpy(), mix[r.rid].omega0.numpy()
        assert np.array_equal(a, m), (r.rid, float(np.abs(a - m).max()))
        assert alone.J_hist == mix[r.rid].J_hist
        assert mix[r.rid].J_hist[-1] < mix[r.rid].J_hist[0]
        w_ref, h_ref, _, _ = _oracle_solve(r)
        assert np.allclose(mix[r.rid].J_hist, h_ref, rtol=1e-9, atol=0), r.rid
        assert rel(m, w_ref) < 1e-9, (r.rid, rel(m, w_ref))
    st = latency_stats(mix)
    assert st["n"] == len(reqs) and st["p99_s"] >= st["p50_s"] > 0


def test_oversize_request_rejected_alone():
    from paper_2602_14016_amd.serving import GpuBackend, Server
    print("CASE serving-reject", flush=True)
    reqs = _make_requests()[:3]
    probe = GpuBackend(slots=1)
    fp = [probe.footprint([r]) for r in reqs]
    assert fp[1] > max(fp[0], fp[2])            # the 64^2 request is the largest
    budget = (fp[1] + max(fp[0], fp[2])) // 2   # fits the 32^2 requests one at a time, never the 64^2 one
    res = Server(hbm_budget_bytes=budget, slots=2).run_trace(reqs)
    assert res[1].status.startswith("rejected")
    assert res[0].status == "ok" and res[2].status == "ok"


def test_cancel_a_running_request():
    """A request cancelled while its batch runs stops at its next iteration boundary: status
    "cancelled", the field of its last completed iteration, fewer iterations than asked."""
    import threading
    import time
    from paper_2602_14016_amd.serving import Server
    print("CASE serving-cancel", flush=True)
    r = _make_requests()[0]
    r.iters, r.arrival = 400, 0.0
    srv = Server(hbm_budget_bytes=8 << 30, slots=1)
    out = {}
    th = threading.Thread(target=lambda: out.update(srv.run_trace([r])))
    th.start()
    t0 = time.time()
    while r.rid not in srv.backend._running and th.is_alive() and time.time() - t0 < 60:
        time.sleep(0.002)
    assert srv.cancel(r.rid)
    th.join(timeout=120)
    assert not th.is_alive()
    res = out[r.rid]
    assert res.status == "cancelled", res.status
    assert 0 <= res.iters < 400 and res.omega0 is not None and torch.isfinite(res.omega0).all()
    assert len(res.J_hist) == res.iters + 1


def test_adaptive_interval_gives_the_same_results():
    """The server's per-group checkpoint interval (the largest its budget share holds) changes
    only how much is recomputed: every request's field and cost history are bitwise those of
    its own interval."""
    from paper_2602_14016_amd.serving import Server
    print("CASE serving-interval", flush=True)
    reqs_a = _make_requests(seed=1)
    reqs_f = _make_requests(seed=1)
    for r in reqs_a + reqs_f:
        r.ckpt_every = 4
    res_a = Server(hbm_budget_bytes=8 << 30, slots=2).run_trace(reqs_a)
    res_f = Server(hbm_budget_bytes=8 << 30, slots=2, adaptive_ckpt=False).run_trace(reqs_f)
    assert any(r.ckpt_every > 4 for r in reqs_a) and all(r.ckpt_every == 4 for r in reqs_f)
    for r in reqs_a:
        a, f = res_a[r.rid], res_f[r.rid]
        assert a.status == f.status == "ok", (a.status, f.status)
        assert torch.equal(a.omega0, f.omega0) and a.J_hist == f.J_hist, r.rid
