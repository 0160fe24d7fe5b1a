"""The serving scheduler on the CPU, with a sleep-model backend in place of the device.

The backend stands for GpuBackend: footprint() sizes a group, run() "solves"
it (sleeps, then returns identifiable host results, a NaN observation making
that member's line search fail as the device solve would), release() frees
it.  The tests check admission by bytes, slot recycling, batching of requests
of one grid and physics whatever their horizons and strides, rejection of
oversize requests, a poisoned request failing alone, an exception failing
only its group, cancellation of a queued request and arrival-order admission
on a Poisson trace.  Requests that must not batch differ in iteration count,
which is part of the batch key.
"""

import threading
import time

import numpy as np
import torch

from paper_2602_14016_amd.serving import Request, Server, latency_stats, poisson_arrivals
from paper_2602_14016_amd.solver import KernelSpec


class SleepBackend:
    def __init__(self, bytes_per_member=100, solve_s=0.05, fail_rids=()):
        self.bytes_per_member = bytes_per_member
        self.solve_s = solve_s
        self.fail_rids = set(fail_rids)
        self.lock = threading.Lock()
        self.active = 0
        self.max_active = 0
        self.calls = []          # (slot, [rids]) in start order
        self.released = []

    def footprint(self, group, ckpt_every=None):
        return self.bytes_per_member * len(group) * (group[0].N // 8)

    def run(self, slot, group, ckpt_every=None):
        with self.lock:
            self.active += 1
            self.max_active = max(self.max_active, self.active)
            self.calls.append((slot, [r.rid for r in group]))
        try:
            time.sleep(self.solve_s)
            if any(r.rid in self.fail_rids for r in group):
                raise RuntimeError("backend failure")
            B, N = len(group), group[0].N
            w = torch.empty((B, N, N), dtype=torch.float64)
            for b, r in enumerate(group):
                w[b].fill_(float(r.rid))
            finite = [bool(torch.isfinite(r.obs_values).all()) for r in group]
            H = [[2.0, 1.0] if ok else [float("nan")] for ok in finite]
            iters = [1 if ok else -1 for ok in finite]     # -(k+1): line search failed after k = 0
            return w, H, iters
        finally:
            with self.lock:
                self.active -= 1

    def release(self, slot, group):
        self.released.append([r.rid for r in group])


def req(rid, arrival=0.0, N=8, n_steps=10, poisoned=False, iters=10, stride=4):
    M = N // stride
    vals = torch.zeros((1, 2, M, M), dtype=torch.float64)
    if poisoned:
        vals[0, 0, 0, 0] = float("nan")
    return Request(rid=rid, N=N, flow="decaying", n_steps=n_steps, stride=stride, obs_steps=[0], obs_values=vals,
                   kernel=KernelSpec(0, 0.0), iters=iters, arrival=arrival)


def test_admission_respects_the_byte_budget_and_recycles_slots():
    be = SleepBackend(bytes_per_member=100, solve_s=0.05)
    # distinct iteration counts: no batching; the budget holds two requests at once although four slots exist
    reqs = [req(i, iters=10 + i) for i in range(6)]
    res = Server(250, slots=4, backend=be).run_trace(reqs)
    assert all(res[r.rid].status == "ok" for r in reqs)
    assert be.max_active == 2
    assert {s for s, _ in be.calls} <= {0, 1, 2, 3}
    assert sorted(sum((c for _, c in be.calls), [])) == list(range(6))
    assert len(be.released) == 6
    be1 = SleepBackend(solve_s=0.02)
    res1 = Server(10 ** 9, slots=2, backend=be1).run_trace([req(i, iters=10 + i) for i in range(5)])
    assert all(r.status == "ok" for r in res1.values())
    assert {s for s, _ in be1.calls} == {0, 1} and be1.max_active <= 2


def test_same_shape_requests_run_as_one_batch_up_to_max_batch():
    be = SleepBackend(solve_s=0.05)
    reqs = [req(i) for i in range(3)]            # one batch key
    res = Server(10 ** 9, slots=1, max_batch=2, backend=be).run_trace(reqs)
    assert [len(c) for _, c in be.calls] == [2, 1]
    assert [res[i].batch for i in range(3)] == [2, 2, 1]
    for i in range(3):
        assert torch.all(res[i].omega0 == float(i))     # each member gets its own result


def test_requests_of_one_grid_batch_across_horizons_and_strides():
    """One grid and physics is one batch, whatever the horizons, strides and kernels; another grid
    or flow is another."""
    be = SleepBackend(solve_s=0.05)
    reqs = [req(0, n_steps=200), req(1, n_steps=1500, stride=2), req(2, N=16, n_steps=300), req(3, n_steps=40)]
    reqs[3].kernel = KernelSpec(2, 0.5)
    res = Server(10 ** 9, slots=1, max_batch=8, backend=be).run_trace(reqs)
    assert [c for _, c in be.calls] == [[0, 1, 3], [2]]
    assert [res[i].batch for i in range(4)] == [3, 3, 1, 3]
    assert all(res[i].status == "ok" for i in range(4))


def test_oversize_request_is_rejected_alone():
    be = SleepBackend(bytes_per_member=100)
    reqs = [req(0), req(1, N=800), req(2, iters=11)]   # request 1 needs 100 * 100 bytes
    res = Server(1000, slots=2, backend=be).run_trace(reqs)
    assert res[1].status.startswith("rejected")
    assert res[0].status == "ok" and res[2].status == "ok"


def test_poisoned_request_fails_alone_inside_a_batch():
    be = SleepBackend()
    reqs = [req(0), req(1, poisoned=True), req(2)]        # one shape, batched together
    res = Server(10 ** 9, slots=1, max_batch=8, backend=be).run_trace(reqs)
    assert [len(c) for _, c in be.calls] == [3]
    assert res[1].status == "line-search failure" and res[1].iters == 0
    assert res[0].status == "ok" and res[2].status == "ok"


def test_backend_exception_fails_only_its_group():
    be = SleepBackend(fail_rids={1})
    reqs = [req(0), req(1, iters=11), req(2, iters=12)]
    res = Server(10 ** 9, slots=2, backend=be).run_trace(reqs)
    assert res[1].status.startswith("error")
    assert res[0].status == "ok" and res[2].status == "ok"
    assert len(be.released) == 3          # the failed group's memory is released too


def test_cancel_a_queued_request():
    be = SleepBackend(solve_s=0.4)
    srv = Server(10 ** 9, slots=1, backend=be)
    reqs = [req(0), req(1, iters=11), req(2, iters=12)]
    out = {}
    th = threading.Thread(target=lambda: out.update(srv.run_trace(reqs)))
    th.start()
    time.sleep(0.15)                      # request 0 is running, 1 and 2 are queued
    assert srv.cancel(1)
    assert not srv.cancel(0)              # already admitted
    assert not srv.cancel(99)
    th.join(timeout=10)
    assert not th.is_alive()
    assert out[1].status == "cancelled"
    assert out[0].status == "ok" and out[2].status == "ok"
    assert [c for _, c in be.calls] == [[0], [2]]


def test_poisson_trace_is_admitted_in_arrival_order():
    arrivals = poisson_arrivals(12, rate=200.0, seed=3)
    assert np.all(np.diff(arrivals) > 0)
    be = SleepBackend(solve_s=0.01)
    reqs = [req(i, arrival=float(a), iters=10 + i) for i, a in enumerate(arrivals)]
    res = Server(10 ** 9, slots=1, backend=be).run_trace(list(reversed(reqs)))
    assert [c[0] for _, c in be.calls] == list(range(12))
    assert all(res[i].admitted >= reqs[i].arrival - 1e-3 for i in range(12))
    st = latency_stats(res)
    assert st["n"] == 12 and st["p99_s"] >= st["p50_s"] > 0


class CancellableSleepBackend(SleepBackend):
    """Solves in 10 ms ticks, one iteration per tick; cancel(rid) stops that member at its next tick."""

    def __init__(self, ticks=40):
        super().__init__(solve_s=0.0)
        self.ticks = ticks
        self.stop = set()
        self.running = set()

    def run(self, slot, group, ckpt_every=None):
        with self.lock:
            self.running |= {r.rid for r in group}
        try:
            done = {r.rid: 0 for r in group}
            for _ in range(self.ticks):
                time.sleep(0.01)
                with self.lock:
                    for r in group:
                        if r.rid not in self.stop:
                            done[r.rid] += 1
            w, H, _ = super().run(slot, group)
            return w, H, [done[r.rid] for r in group]
        finally:
            with self.lock:
                self.running -= {r.rid for r in group}

    def cancel(self, rid):
        with self.lock:
            if rid not in self.running:
                return False
            self.stop.add(rid)
            return True


def test_cancel_a_running_request_stops_it_alone():
    be = CancellableSleepBackend(ticks=40)
    srv = Server(10 ** 9, slots=1, max_batch=8, backend=be)
    reqs = [req(0), req(1)]        # one shape: one batch
    for r in reqs:
        r.iters = 40
    out = {}
    th = threading.Thread(target=lambda: out.update(srv.run_trace(reqs)))
    th.start()
    t0 = time.time()
    while not be.running and time.time() - t0 < 5:
        time.sleep(0.005)
    time.sleep(0.05)
    assert srv.cancel(1)
    th.join(timeout=10)
    assert not th.is_alive()
    assert out[1].status == "cancelled" and 0 < out[1].iters < 40
    assert out[0].status == "ok" and out[0].iters == 40
    assert not srv.cancel(1) and not srv.cancel(0)        # finished


class IntervalBackend(SleepBackend):
    """Footprint grows with the checkpoint interval, as the segment store does."""

    def footprint(self, group, ckpt_every=None):
        K = group[0].ckpt_every if ckpt_every is None else ckpt_every
        return len(group) * (1000 + 10 * K)

    def run(self, slot, group, ckpt_every=None):
        with self.lock:
            self.intervals = getattr(self, "intervals", []) + [(group[0].rid, ckpt_every)]
        return super().run(slot, group, ckpt_every)


def test_admitted_groups_get_the_largest_interval_that_fits():
    be = IntervalBackend(solve_s=0.01)
    # budget 40000 over 2 slots: share 20000 -> 1000 + 10 K <= 20000 -> K = 1900 for one member
    reqs = [req(0, n_steps=5000), req(1, n_steps=300, iters=11), req(2, n_steps=40, iters=12)]
    for r in reqs:
        r.ckpt_every = 50
    res = Server(40000, slots=2, backend=be).run_trace(reqs)
    assert all(r.status == "ok" for r in res.values())
    got = dict(be.intervals)
    assert got[0] == 1900            # the largest that fits the slot's share
    assert got[1] == 300             # the whole horizon fits
    assert got[2] == 50              # the own interval already covers the horizon
    be2 = IntervalBackend(solve_s=0.01)
    r = req(3, n_steps=5000)
    r.ckpt_every = 50
    Server(40000, slots=2, backend=be2, adaptive_ckpt=False).run_trace([r])
    assert dict(be2.intervals)[3] == 50


def test_groups_are_trimmed_until_their_interval_covers_half_the_horizon():
    """A group whose checkpoint interval would fall below half its horizon (a recomputation sweep
    over most of it) loses its latest arrivals until the interval fits or one member is left."""
    be = IntervalBackend(solve_s=0.01)
    # share 20000 per slot: B members fit an interval K <= 20000 / B / 10 - 100
    long = [req(i, n_steps=2000) for i in range(4)]        # B = 4 gives K = 400 < 1000: run one by one
    short = [req(10 + i, n_steps=800, iters=11) for i in range(4)]   # B = 4 gives K = 400 = 800 / 2: one batch
    for r in long + short:
        r.ckpt_every = 50
    res = Server(40000, slots=2, max_batch=8, backend=be, min_interval_frac=0.5).run_trace(long + short)
    assert all(r.status == "ok" for r in res.values())
    assert [res[i].batch for i in range(4)] == [1, 1, 1, 1]
    assert [res[10 + i].batch for i in range(4)] == [4, 4, 4, 4]
    got = dict(be.intervals)
    assert got[0] == 1900 and got[10] == 400
