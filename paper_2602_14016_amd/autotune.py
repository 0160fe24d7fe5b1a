"""Autotuner for the FFT tile shapes of a Solver.

Knobs (pa_set_tiles), one set per pass: the register plan of the 1D
transforms (variant 0: more elements per thread; 1: more threads per
transform; 2: four elements per thread where the length allows; 3, row
passes only: variant 2's plan in persistent wavefronts that prefetch their
next rows into LDS) and the workgroup shape (rows per workgroup for the forward and the adjoint row
passes, kx columns per workgroup for the column pass), and for the column
pass the number of workgroups that share out each column's output transforms
(0: chosen per launch from the wavefronts it has; 1, 2 or 4 fixed).  The three passes are
separate kernels reading and writing fixed layouts, so each is tuned on its
own: every candidate runs a short batched forward + adjoint solve of the
solver's own shape while the library times that pass's launches with HIP
events on the solver's stream (pa_profile_start).  Forward rows are scored by
the right-hand-side row kernel, adjoint rows by the adjoint-product row
kernel, and the column pass by its forward plus adjoint stage launches; for
the column pass every (variant, block) pair is tried with each share count,
since the best count depends on the block (wide blocks fill a CU alone and
want fewer shares).  The best of each is applied and returned.  Results depend on the choice only through the
rounding of the transforms (not at all on the column shares).
"""

import time

import torch

ROW_VARIANTS = (0, 1, 2, 3)
COL_VARIANTS = (0, 1, 2)
BLOCKS = (1, 2, 4, 8)
COL_SPLITS = (0, 1, 2, 4)
ROW_NL, COL_FWD, ROW_ADJ, COL_ADJ = 0, 1, 2, 3


def _class_cost(solver, omega0, n_steps, classes, reps):
    """Total device time (ms) of the launches of `classes` in one solve (min over reps)."""
    n = solver.N
    best = None
    for _ in range(reps):
        total = 0.0
        for cls in classes:
            solver.profile_start(cls, 1)
            solver.adjoint_impulse(omega0, n_steps, n // 2, n // 2, 1, ckpt_every=n_steps)
            p = solver.profile_stop()
            total += p["total_ms"] / max(p["timed_launches"], 1) * p["launches"]
        best = total if best is None else min(best, total)
    return best


def _time_solve(solver, omega0, n_steps, reps):
    stream = torch.cuda.current_stream(solver.device)
    n = solver.N
    solver.adjoint_impulse(omega0, n_steps, n // 2, n // 2, 1, ckpt_every=n_steps)   # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        solver.adjoint_impulse(omega0, n_steps, n // 2, n // 2, 1, ckpt_every=n_steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(solver, omega0=None, n_steps=8, reps=2, verbose=False):
    """Pick the tiles of every pass for `solver`, apply them; returns a dict."""
    if omega0 is None:
        omega0 = solver.init_field(list(range(solver.B)), kind=0, k0=max(2.0, solver.N / 25), target=0.5)
    t_start = time.perf_counter()
    trials = []
    chosen = {}
    searches = (
        ("row", ROW_VARIANTS, "row_variant", "row_teams", (ROW_NL,)),
        ("adj", ROW_VARIANTS, "adj_variant", "adj_teams", (ROW_ADJ,)),
        ("col", COL_VARIANTS, "col_variant", "col_block", (COL_FWD, COL_ADJ)),
    )
    solver.set_tiles(col_split=0)
    for name, variants, vkey, bkey, classes in searches:
        splits = COL_SPLITS if name == "col" else (None,)
        best = None
        for v in variants:
            for blk in BLOCKS:
                try:
                    solver.set_tiles(**{vkey: v, bkey: blk})
                except Exception:
                    continue
                for sp in splits:
                    if sp is not None:
                        solver.set_tiles(col_split=sp)
                    ms = _class_cost(solver, omega0, n_steps, classes, reps)
                    trials.append({"pass": name, "variant": v, "block": blk, "ms": ms}
                                  | ({} if sp is None else {"split": sp}))
                    if best is None or ms < best[0]:
                        best = (ms, v, blk, sp)
        chosen[vkey], chosen[bkey] = best[1], best[2]
        solver.set_tiles(**{vkey: best[1], bkey: best[2]})
        if best[3] is not None:
            chosen["col_split"] = best[3]
            solver.set_tiles(col_split=best[3])
    out = dict(solver.get_tiles())
    out["ms"] = _time_solve(solver, omega0, n_steps, reps)
    out["trials"] = trials
    out["seconds"] = time.perf_counter() - t_start
    out["probe"] = f"{solver.B} x {solver.N}^2, {n_steps} forward + {n_steps} adjoint steps"
    if verbose:
        for r in trials:
            print("autotune", r)
        print("autotune best", {k: out[k] for k in chosen} | {"ms": out["ms"]})
    return out
