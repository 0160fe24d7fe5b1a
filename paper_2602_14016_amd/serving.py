"""Continuous-batching request server for assimilation solves.

Requests (grid size, flow, horizon, observation stride and steps, kernel,
iteration count, observations) arrive over time.  The server keeps a queue
and a fixed number of slots; each slot owns a HIP stream (default priority)
and a worker thread.  Whenever a slot is free, queued requests are admitted in
arrival order if their device footprint (workspace + fields + observations,
from pa_workspace_bytes) fits in the remaining HBM budget.  Waiting requests
of the same grid and flow physics (and iteration count) are admitted
together as one batched solve, whatever their horizons, probe strides,
observation times and kernels: pa_assimilate_members gives every member its
own observation set, and a member advances only through its own horizon, so
batching costs no padded work.  A slot uploads the group's observations,
forms each request's first guess, runs the solve on its stream and copies the
results back; its memory is released for the next admission as soon as it
finishes.  Each admitted group gets the largest checkpoint interval that fits
its slot's share of the budget, so gradients recompute fewer segments (none
when the whole trajectory fits); results do not depend on it.  Solves on
different slots overlap on the device.  Latency is stamped from arrival to
result-ready.

Results of a request are identical whether it runs alone, batched with
others or concurrently with other slots: every member uses the same kernels
with the same tiles (a fixed table per grid size, never chosen per batch),
no reduction crosses members, and a member's steps are those of its own
horizon.

    python -m paper_2602_14016_amd.serving --requests R --rate HZ [--load F] --out FILE

replays a seeded Poisson trace of the mixed workload (grids 128..1024,
decaying and Kolmogorov flow, horizons 200..2000, strides 4..16, mixed
kernels, 10 L-BFGS iterations each) and prints p50/p99 latency and
throughput; with --load F a second trace runs at F times the capacity the
first one measured.
"""

import heapq
import queue
import threading
import time
from dataclasses import dataclass, replace, field
from typing import List, Optional

import numpy as np
import torch

from .solver import KernelSpec, Observations, Solver

DECAYING = "decaying"
KOLMOGOROV = "kolmogorov"


def physics_for(flow, N):
    """Per-flow physics: decaying HIT (nu = 1e-4) or Kolmogorov (nu = 1/40, drag 0.1, A = 1, n_f = 4),
    with a time step that keeps the explicit nonlinear term stable at grid size N."""
    if flow == DECAYING:
        dt = 2e-3 if N <= 256 else (1e-3 if N == 512 else 5e-4)
        return dict(nu=1e-4, mu=0.0, dt=dt, forcing_amp=0.0, forcing_k=4)
    dt = 1e-3 if N <= 512 else 5e-4
    return dict(nu=1.0 / 40, mu=0.1, dt=dt, forcing_amp=1.0, forcing_k=4)


@dataclass
class Request:
    rid: int
    N: int
    flow: str
    n_steps: int
    stride: int
    obs_steps: List[int]
    obs_values: torch.Tensor          # host float64 [n_times, 2, M, M]
    kernel: KernelSpec
    iters: int = 10
    lbfgs_m: int = 10
    ckpt_every: int = 50
    first_guess: str = "interp"       # "interp" (spectral interpolation of t=0 probes) or "zero"
    arrival: float = 0.0              # seconds from trace start

    def batch_key(self):
        """Requests with equal keys run as one batched solve: one grid and physics, one iteration
        count and memory; horizons, strides, observation times and kernels may differ."""
        return (self.N, self.flow, self.iters, self.lbfgs_m, self.first_guess)


@dataclass
class Result:
    rid: int
    omega0: Optional[torch.Tensor]
    J_hist: List[float]
    iters: int
    status: str
    arrival: float
    admitted: float
    finished: float
    batch: int

    @property
    def latency(self):
        return self.finished - self.arrival


def group_shape(group):
    """(horizon, most observation times) of a batched group: its solve runs to the longest horizon."""
    return max(r.n_steps for r in group), max(len(r.obs_steps) for r in group)


def footprint_bytes(solver, group, ckpt_every):
    """Device bytes of a group's solve: the workspace at the group's longest horizon and largest
    observation count, plus each member's field, first guess, result and observations."""
    H, n_obs = group_shape(group)
    m = max(max(r.lbfgs_m for r in group), 1)
    ws = solver.workspace_bytes(H, ckpt_every, n_obs, m)
    N = group[0].N
    fields = sum((3 * N * N + len(r.obs_steps) * 2 * (N // r.stride) ** 2) * 8 for r in group)
    return ws + fields


class GpuBackend:
    """The device work of the server: one HIP stream (default priority) per slot.
    footprint() sizes a group from a sizing context per (grid, batch size) that only
    the scheduler thread uses; run() creates the group's contexts on its slot's stream,
    assimilates the group as one batched solve and returns host results; release()
    frees the group's contexts and workspace."""

    def __init__(self, slots, device="cuda:0", tiles=None):
        self.device = torch.device(device)
        self.tiles = dict(tiles or {})
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self._sizing = {}    # (N, B) -> Solver, scheduler thread only (workspace-size queries)
        self._live = {}      # slot -> Solvers of the group running there
        self._lock = threading.Lock()
        self._running = {}   # rid -> (cancel flags of its solver, member index)

    def _new_solver(self, slot, N, flow, B):
        with torch.cuda.stream(self.streams[slot]):
            sv = Solver(N, B, device=self.device, stream=self.streams[slot], **physics_for(flow, N))
        if N in self.tiles:
            sv.set_tiles(**self.tiles[N])
        return sv

    def footprint(self, group, ckpt_every=None):
        """Device bytes of running `group` (requests of one batch key) with checkpoints every
        ckpt_every steps (default: the head's own interval)."""
        head = group[0]
        key = (head.N, len(group))
        if key not in self._sizing:
            self._sizing[key] = Solver(head.N, len(group), device=self.device, **physics_for(DECAYING, head.N))
        K = head.ckpt_every if ckpt_every is None else ckpt_every
        return footprint_bytes(self._sizing[key], group, K)

    def run(self, slot, group, ckpt_every=None):
        """(omega0 [B, N, N] on the host, J histories, iteration counts) of the group, in its order."""
        head = group[0]
        B = len(group)
        K = head.ckpt_every if ckpt_every is None else ckpt_every
        # longest horizon first: at every step the members still advancing share one launch
        order = sorted(range(B), key=lambda i: -group[i].n_steps)
        g = [group[i] for i in order]
        s = self._new_solver(slot, head.N, head.flow, B)
        one = self._new_solver(slot, head.N, head.flow, 1)   # first guesses, member by member
        self._live[slot] = (s, one)
        with torch.cuda.stream(self.streams[slot]):
            obs, fg = [], torch.zeros((B, head.N, head.N), dtype=torch.float64, device=self.device)
            for b, r in enumerate(g):
                vals = r.obs_values.to(self.device, dtype=torch.float64, non_blocking=False).contiguous()[None]
                obs.append(Observations(r.stride, r.obs_steps, vals))
                if r.first_guess == "interp" and r.obs_steps and r.obs_steps[0] == 0:
                    fg[b] = one.first_guess(r.stride, vals[:, 0].contiguous())[0]
            flags = s.cancel_flags()
            with self._lock:
                for b, r in enumerate(g):
                    self._running[r.rid] = (flags, b)
            try:
                w, H, iters = s.assimilate_members(fg, obs, [r.kernel for r in g], "lbfgs", head.iters,
                                                   head.lbfgs_m, K)
            finally:
                with self._lock:
                    for r in g:
                        self._running.pop(r.rid, None)
            w = w.cpu()
        back = [0] * B
        for b, i in enumerate(order):
            back[i] = b
        return w[back], [H[back[i]] for i in range(B)], [iters[back[i]] for i in range(B)]

    def cancel(self, rid):
        """Stop a running request at its next iteration boundary; False if it is not running."""
        with self._lock:
            hit = self._running.get(rid)
            if hit is None:
                return False
            flags, b = hit
            flags[b] = 1
            return True

    def release(self, slot, group):
        for sv in self._live.pop(slot, ()):
            sv._ws = None   # return the workspace to the allocator before the budget is released
            sv.close()
        # ... and its segments to the device: a cached workspace (tens of GB) would otherwise
        # be split to serve smaller blocks and could no longer be handed back whole, so the
        # next large workspace fails with most of the memory reserved but unused
        torch.cuda.empty_cache()


class Server:
    def __init__(self, hbm_budget_bytes, slots=4, max_batch=8, device="cuda:0", tiles=None, verbose=False,
                 backend=None, adaptive_ckpt=True, min_interval_frac=0.0):
        """tiles: optional {N: pa_tiles dict} applied to every solver of grid size N;
        verbose: print one line per finished group; backend: the device work
        (GpuBackend by default; anything with footprint/run/release);
        adaptive_ckpt: give each admitted group the largest checkpoint interval
        that fits its share of the budget (fewer recomputed segments, the same
        result bit for bit) instead of the requests' own; min_interval_frac: a group is
        trimmed (latest arrivals first) until its checkpoint interval covers at least this
        fraction of its horizon, so that batching never buys its per-member efficiency with
        a recomputation sweep over most of the horizon (at 1024^2 a member's whole
        trajectory is tens of GB, and eight of them would leave segments of a few dozen
        steps)."""
        self.backend = backend if backend is not None else GpuBackend(slots, device, tiles)
        self.verbose = verbose
        self.budget = int(hbm_budget_bytes)
        self.in_use = 0
        self.slots = slots
        self.max_batch = max_batch
        self.lock = threading.Condition()
        self.queue: List[Request] = []
        self.results = {}
        self.cancelled = set()   # running requests asked to stop
        self.adaptive_ckpt = adaptive_ckpt
        self.min_interval_frac = float(min_interval_frac)
        self.free_slots = list(range(slots))
        self.t0 = None

    # ------------------------------------------------------------------ API
    def now(self):
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        with self.lock:
            self.queue.append(req)
            self.lock.notify_all()

    def cancel(self, rid):
        """Withdraw a queued request, or stop a running one at its next iteration boundary (its
        result is then the last completed iterate, status "cancelled"; the other requests of its
        batch run on unchanged).  False if it is finished, unknown, or the backend cannot stop
        a running solve."""
        with self.lock:
            for r in self.queue:
                if r.rid == rid:
                    self.queue.remove(r)
                    t = self.now() if self.t0 is not None else 0.0
                    self.results[rid] = Result(rid, None, [], 0, "cancelled", r.arrival, t, t, 0)
                    self.lock.notify_all()
                    return True
            stop = getattr(self.backend, "cancel", None)
            if stop is not None and rid not in self.results and stop(rid):
                self.cancelled.add(rid)
                return True
        return False

    def _admit_locked(self):
        """Admit queued requests into free slots while memory allows (arrival order): the oldest
        request and the waiting requests of its batch key, up to max_batch, as one group."""
        started = []
        while self.free_slots and self.queue:
            head = self.queue[0]
            group = [r for r in self.queue if r.batch_key() == head.batch_key()][: self.max_batch]
            need = self.backend.footprint(group)
            while need > self.budget - self.in_use and len(group) > 1:
                group = group[:-1]
                need = self.backend.footprint(group)
            if need > self.budget:
                self.queue.remove(head)
                self.results[head.rid] = Result(head.rid, None, [], 0, "rejected: exceeds HBM budget",
                                                head.arrival, self.now(), self.now(), 0)
                continue
            if need > self.budget - self.in_use:
                break   # wait for memory to free up
            K = self._interval(group)
            while (self.adaptive_ckpt and len(group) > 1
                   and K < self.min_interval_frac * max(r.n_steps for r in group)):
                group = group[:-1]
                K = self._interval(group)
            need = self.backend.footprint(group, K)
            for r in group:
                self.queue.remove(r)
            slot = self.free_slots.pop(0)
            self.in_use += need
            started.append((slot, group, need, K))
        return started

    def _interval(self, group):
        """The largest checkpoint interval, from the requests' own up to the group's whole horizon,
        whose footprint fits this slot's share of the budget and the memory free now.  A longer
        interval recomputes fewer segments in every gradient (none once the whole trajectory is
        kept), and the solve's result does not depend on it.  The footprint grows with the
        interval (the segment store dominates), so a bisection finds it."""
        head = group[0]
        H = max(r.n_steps for r in group)
        own = max(1, min(head.ckpt_every, H))
        if not self.adaptive_ckpt or H <= own:
            return head.ckpt_every
        share = min(self.budget // self.slots, self.budget - self.in_use)
        fits = lambda k: self.backend.footprint(group, k) <= share
        if fits(H):
            return H
        lo, hi = own, H                   # lo: the requests' own interval or one that fits
        while hi - lo > 1:
            mid = (lo + hi) // 2
            if fits(mid):
                lo = mid
            else:
                hi = mid
        return lo

    def _run_group(self, slot, group, need, K):
        admitted = self.now()
        try:
            head = group[0]
            B = len(group)
            for r in group:
                r.ckpt_every = K
            w_host, H, iters = self.backend.run(slot, group, K)
            fin = self.now()
            if self.verbose:
                print(f"[serving] slot {slot}: {B} x {head.N}^2 {head.flow} H={[r.n_steps for r in group]} K={K} "
                      f"done at {fin:.2f} s (admitted {admitted:.2f} s)", flush=True)
            for b, r in enumerate(group):
                status = "ok" if iters[b] >= 0 else "line-search failure"
                if r.rid in self.cancelled and iters[b] >= 0 and iters[b] < r.iters:
                    status = "cancelled"
                self.results[r.rid] = Result(r.rid, w_host[b].clone(), [h for h in H[b] if h == h],
                                             iters[b] if iters[b] >= 0 else -iters[b] - 1, status, r.arrival,
                                             admitted, fin, B)
        except Exception as e:   # a failing request fails alone
            fin = self.now()
            for r in group:
                self.results[r.rid] = Result(r.rid, None, [], 0, f"error: {e}", r.arrival, admitted, fin, len(group))
        finally:
            try:
                self.backend.release(slot, group)
            except Exception:
                pass
            with self.lock:
                self.in_use -= need
                self.free_slots.append(slot)
                self.free_slots.sort()
                self.lock.notify_all()

    def run_trace(self, requests: List[Request], time_scale=1.0):
        """Replay requests at their arrival times (seconds * time_scale); returns results by id."""
        self.t0 = time.perf_counter()
        pending = sorted(requests, key=lambda r: r.arrival)
        threads = []
        i = 0
        while True:
            now = self.now()
            while i < len(pending) and pending[i].arrival * time_scale <= now:
                self.submit(pending[i])
                i += 1
            with self.lock:
                started = self._admit_locked()
            for slot, group, need, K in started:
                th = threading.Thread(target=self._run_group, args=(slot, group, need, K), daemon=True)
                th.start()
                threads.append(th)
            with self.lock:
                done = i == len(pending) and not self.queue and len(self.free_slots) == self.slots
                if done:
                    break
                next_arrival = pending[i].arrival * time_scale - self.now() if i < len(pending) else None
                timeout = 0.05 if next_arrival is None else max(0.0, min(0.05, next_arrival))
                self.lock.wait(timeout=timeout)
        for th in threads:
            th.join()
        return dict(self.results)


def poisson_arrivals(n, rate, seed=0):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def latency_stats(results):
    lat = sorted(r.latency for r in results.values() if r.status == "ok")
    if not lat:
        return {}
    q = lambda p: float(np.percentile(np.array(lat), p))
    return {"n": len(lat), "p50_s": q(50), "p99_s": q(99), "mean_s": float(np.mean(lat)), "max_s": lat[-1]}


# ------------------------------------------------------------ trace CLI --

GRIDS = (128, 256, 512, 1024)
KERNELS = (KernelSpec(0, 0.0), KernelSpec(1, 0.05), KernelSpec(2, 0.5))


def make_trace(n, rate, seed=0, iters=10, grids=GRIDS, h_range=(200, 2000), strides=(4, 8, 16), device="cuda:0"):
    """Seeded mixed requests with Poisson arrivals; observations (5 evenly spaced
    times from step 0) come from a truth run of another seed, computed here,
    before the trace, and kept on the host."""
    rng = np.random.default_rng(seed)
    arrivals = poisson_arrivals(n, rate, seed=seed + 1)
    reqs = []
    for i in range(n):
        N = int(rng.choice(grids))
        flow = DECAYING if rng.random() < 0.5 else KOLMOGOROV
        H = int(rng.integers(h_range[0], h_range[1] + 1))
        stride = int(rng.choice(strides))
        kern = KERNELS[int(rng.integers(len(KERNELS)))]
        steps = sorted({int(round(j * H / 4)) for j in range(5)})
        truth_solver = Solver(N, 1, device=device, **physics_for(flow, N))
        truth = truth_solver.init_field([1000 + i], kind=0 if flow == DECAYING else 2, k0=max(2.0, N / 25),
                                        target=0.5 if flow == DECAYING else 1e-2)
        obs = truth_solver.forward(truth, H, Observations(stride, steps), want_obs=True)["obs"][0].cpu()
        truth_solver.close()
        reqs.append(Request(rid=i, N=N, flow=flow, n_steps=H, stride=stride, obs_steps=steps, obs_values=obs,
                            kernel=kern, iters=iters, arrival=float(arrivals[i])))
    return reqs


def tile_table(grids=GRIDS, device="cuda:0", batch=4):
    """One autotuned tile set per grid size, fixed for the whole trace so that a request's result
    does not depend on its batch (the plan variants set the rounding).  It is tuned on a batch of
    `batch` members, the size the groups of a loaded server run at (tuned on one member, the
    1024^2 set took the one-wavefront adjoint-row plan and wide column blocks, 25-40 % slower per
    launch at four to eight members); the column share count is left to each launch (0), which
    gives one-member launches their shares."""
    from .autotune import autotune
    table = {}
    for N in grids:
        sv = Solver(N, batch, device=device, **physics_for(DECAYING, N))
        autotune(sv, n_steps=4)
        table[N] = sv.get_tiles() | {"col_split": 0}
        sv.close()
    return table


def trace_report(results, requests, t_wall):
    ok = [r for r in results.values() if r.status == "ok"]
    work = sum(q.N * q.N * q.n_steps for q in requests if results[q.rid].status == "ok")
    out = latency_stats(results)
    statuses = {}
    for r in results.values():
        statuses[r.status] = statuses.get(r.status, 0) + 1
    out.update({"requests": len(requests), "completed": len(ok), "wall_s": t_wall,
                "throughput_req_per_s": len(ok) / t_wall if t_wall > 0 else None,
                "grid_point_steps_per_iteration_per_s": work * (requests[0].iters if requests else 0) / t_wall,
                "batched_solves": sum(1 for r in ok if r.batch > 1), "statuses": statuses,
                "not_ok": [[q.rid, q.N, q.flow, q.n_steps, q.ckpt_every, results[q.rid].status]
                           for q in requests if results[q.rid].status != "ok"],
                "intervals": [[q.rid, q.N, q.n_steps, q.ckpt_every] for q in requests]})
    return out


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--requests", type=int, default=40)
    ap.add_argument("--rate", type=float, default=20.0, help="arrivals per second")
    ap.add_argument("--load", type=float, default=0.0, help="also replay at this fraction of measured capacity")
    ap.add_argument("--iters", type=int, default=10)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fixed-ckpt", action="store_true",
                    help="keep each request's own checkpoint interval (50) instead of the largest that fits")
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)
    tiles = tile_table()
    print("tiles", json.dumps({str(k): v for k, v in tiles.items()}), flush=True)
    report = {"tiles": {str(k): v for k, v in tiles.items()}, "traces": []}
    rate = args.rate
    for label in ("offered", "capacity") if args.load > 0 else ("offered",):
        reqs = make_trace(args.requests, rate, seed=args.seed, iters=args.iters)
        print(f"trace {label}: {len(reqs)} requests at {rate:.2f}/s", flush=True)
        srv = Server(int(args.budget_gb * (1 << 30)), slots=args.slots, max_batch=args.max_batch, tiles=tiles,
                     verbose=True, adaptive_ckpt=not args.fixed_ckpt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run_trace(reqs)
        t_wall = time.perf_counter() - t0
        rep = trace_report(res, reqs, t_wall)
        rep.update({"trace": label, "rate_per_s": rate})
        print(json.dumps(rep), flush=True)
        report["traces"].append(rep)
        if label == "offered" and args.load > 0:
            busy = max(r.finished for r in res.values()) - min(r.admitted for r in res.values())
            capacity = rep["completed"] / busy if busy > 0 else rate
            rate = args.load * capacity
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(report, fh, indent=1)


if __name__ == "__main__":
    main()
