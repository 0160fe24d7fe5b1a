"""Autotuner for the FFT tile shapes of a Solver.

Knobs (pa_set_tiles): the register plan of the 1D transforms (variant 0:
more elements per thread; 1: more threads per transform), the number of kx
columns per column-pass workgroup, and the number of rows per row-pass
workgroup.  Each candidate is timed with HIP events on a short batched
forward + adjoint solve of the solver's own shape (the same kernels the real
solve runs); the fastest is applied and returned.  Results depend on the
choice only through the rounding of the transforms.
"""

import itertools
import time

import torch


def _time_solve(solver, omega0, n_steps, ckpt_every, reps):
    stream = torch.cuda.current_stream(solver.device)
    n = solver.N
    solver.adjoint_impulse(omega0, n_steps, n // 2, n // 2, 1, ckpt_every=ckpt_every)   # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        solver.adjoint_impulse(omega0, n_steps, n // 2, n // 2, 1, ckpt_every=ckpt_every)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def candidates(N):
    variants = [0, 1]
    cbs = [1, 2, 4, 8]
    tpbs = [1, 2, 4, 8]
    return variants, cbs, tpbs


def autotune(solver, omega0=None, n_steps=16, ckpt_every=8, reps=2, verbose=False):
    """Pick (fft_variant, col_block, row_teams) for `solver`; returns a dict."""
    if omega0 is None:
        omega0 = solver.init_field(list(range(solver.B)), kind=0, k0=max(2.0, solver.N / 25), target=0.5)
    variants, cbs, tpbs = candidates(solver.N)
    results = []
    best = None
    t_start = time.perf_counter()
    for var in variants:
        # column block first (row teams at 4), then row teams with the best column block
        local = None
        for cb in cbs:
            try:
                solver.set_tiles(cb, 4, var)
            except Exception:
                continue
            ms = _time_solve(solver, omega0, n_steps, ckpt_every, reps)
            results.append({"fft_variant": var, "col_block": cb, "row_teams": 4, "ms": ms})
            if local is None or ms < local[0]:
                local = (ms, cb, 4)
        if local is None:
            continue
        for tpb in tpbs:
            if tpb == 4:
                continue
            solver.set_tiles(local[1], tpb, var)
            ms = _time_solve(solver, omega0, n_steps, ckpt_every, reps)
            results.append({"fft_variant": var, "col_block": local[1], "row_teams": tpb, "ms": ms})
            if ms < local[0]:
                local = (ms, local[1], tpb)
        if best is None or local[0] < best[0]:
            best = (local[0], local[1], local[2], var)
    solver.set_tiles(best[1], best[2], best[3])
    out = {"fft_variant": best[3], "col_block": best[1], "row_teams": best[2], "ms": best[0],
           "trials": results, "seconds": time.perf_counter() - t_start,
           "probe": f"{solver.B} x {solver.N}^2, {n_steps} forward + {n_steps} adjoint steps"}
    if verbose:
        for r in results:
            print("autotune", r)
        print("autotune best", {k: out[k] for k in ("fft_variant", "col_block", "row_teams", "ms")})
    return out
