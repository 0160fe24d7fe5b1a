"""Autotuner for the FFT tile shapes of a Solver.

Knobs (pa_set_tiles): the register plan of the 1D transforms of the row
passes and of the column pass (variant 0: more elements per thread; 1: more
threads per transform; 2: four elements per thread where the length allows),
the number of rows per row-pass workgroup and the number of kx columns per
column-pass workgroup.  Each candidate is timed with HIP events on a short
batched forward + adjoint solve of the solver's own shape (the same kernels
the real solve runs).  The row and column passes are separate kernels, so the
search is coordinate-wise: row plan and rows per workgroup first (column
tiles at their defaults), then column plan and columns per workgroup with the
best row tiles.  The fastest is applied and returned.  Results depend on the
choice only through the rounding of the transforms.
"""

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


VARIANTS = (0, 1, 2)
BLOCKS = (1, 2, 4, 8)


def autotune(solver, omega0=None, n_steps=16, ckpt_every=8, reps=2, verbose=False):
    """Pick (row_variant, row_teams, col_variant, col_block) for `solver`; returns a dict."""
    if omega0 is None:
        omega0 = solver.init_field(list(range(solver.B)), kind=0, k0=max(2.0, solver.N / 25), target=0.5)
    results = []
    t_start = time.perf_counter()

    def trial(rv, tpb, cv, cb):
        try:
            solver.set_tiles(cb, tpb, rv, cv)
        except Exception:
            return None
        ms = _time_solve(solver, omega0, n_steps, ckpt_every, reps)
        results.append({"row_variant": rv, "row_teams": tpb, "col_variant": cv, "col_block": cb, "ms": ms})
        return ms

    best = None
    for rv in VARIANTS:
        for tpb in BLOCKS:
            ms = trial(rv, tpb, 1, 8)
            if ms is not None and (best is None or ms < best[0]):
                best = (ms, rv, tpb, 1, 8)
    _, rv, tpb, _, _ = best
    for cv in VARIANTS:
        for cb in BLOCKS:
            if (cv, cb) == (best[3], best[4]):
                continue
            ms = trial(rv, tpb, cv, cb)
            if ms is not None and ms < best[0]:
                best = (ms, rv, tpb, cv, cb)
    ms, rv, tpb, cv, cb = best
    solver.set_tiles(cb, tpb, rv, cv)
    out = {"row_variant": rv, "row_teams": tpb, "col_variant": cv, "col_block": cb, "ms": ms,
           "trials": results, "seconds": time.perf_counter() - t_start,
           "probe": f"{solver.B} x {solver.N}^2, {n_steps} forward + {n_steps} adjoint steps"}
    if verbose:
        for r in results:
            print("autotune", r)
        print("autotune best", {k: out[k] for k in ("row_variant", "row_teams", "col_variant", "col_block", "ms")})
    return out
