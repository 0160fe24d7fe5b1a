#!/usr/bin/env python
"""Benchmark of the hot path on one MI355X.

One step = one complete batched forward + adjoint solve of the ensemble
workload: 64 independent realizations of 256^2 decaying 2D turbulence (k0 =
10 random-phase spectrum, energy 0.5, seeds 0..63), nu = 1e-4, dt = 2e-3,
500 forward steps, 500 adjoint steps from a unit u-impulse at (128, 128),
per-shell adjoint energy for |k| in 1..85 after every adjoint step.  The
checkpoint interval defaults to the largest whose workspace fits in free HBM:
on a 288 GB device the whole stage trajectory of the 64 members (about 185 GB)
stays resident, so the adjoint needs no recomputation (--ckpt-every 50 gives
the checkpointed form).  Inputs are resident in HBM before the timed region.  value = members * N^2 * horizon * steps / seconds
(grid-point-steps/s, each unit one point advanced one forward and one adjoint
step).  Beside it: the plain path (one member per solve, same kernels, the
batch's members solved one after another: equal work), p50/p99 solve latency, the roofline of the dominant kernel measured with HIP
events on its stream, the solve replayed from a captured HIP graph, the same
solve with checkpoints every 50 steps (forward, segment recomputation and
adjoint), a short serving trace of the mixed request workload (p50/p99
latency and throughput, offered at 20 requests/s and then at 0.8 of the
capacity that trace measured), and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "grid-point-steps/s fwd+adj FP64, batched vs plain at 256²; p50/p99 solve latency"

def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * p / 100.0
    lo = int(k)
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(N, nu, dt, steps_sample, k0):
    """The oracle as written (NumPy, its own DFT), one member, a short horizon."""
    import numpy as np
    import oracle as O
    from oracle.model import Physics
    threads = None
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 0) for p in threadpool_info()), default=None)
    except Exception:
        pass
    ph = Physics(N=N, nu=nu, dt=dt)
    w0 = O.init_field(N, [0], kind=0, k0=k0, target=0.5)[0]
    t0 = time.perf_counter()
    O.impulse_adjoint(w0, ph, steps_sample, N // 2, N // 2, (N - 1) // 3)
    t = time.perf_counter() - t0
    return {"value": N * N * steps_sample / t, "unit": "grid-point-steps/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"1 member, {N}^2, {steps_sample} forward + {steps_sample} adjoint steps of the same "
                      f"impulse-response solve (NumPy oracle with exact-twiddle DFT matrices), {t:.1f} s"}


def serving_leg(n_requests, load, device):
    """The mixed request workload (grids 128..1024, decaying and Kolmogorov flow, horizons
    200..2000, strides 4..16, three kernels, 10 L-BFGS iterations each): a trace of n_requests
    Poisson arrivals at 20/s (the offered rate; the queue grows), then the same requests at
    `load` times the capacity it measured.  Tiles are autotuned per grid before the traces."""
    import dataclasses
    import numpy as np
    import torch
    from paper_2602_14016_amd import serving as sv
    tiles = sv.tile_table(device=device)
    reqs = sv.make_trace(n_requests, 20.0, seed=0, device=device)
    out = {"requests": n_requests, "workload": "mixed requests: grids 128..1024, decaying and Kolmogorov flow, "
           "horizons 200..2000, strides 4..16, kernels identity / exp(-0.05|k|) / |k|^-1, 10 L-BFGS iterations "
           "each, 4 slots, 200 GB budget", "traces": []}
    rate = 20.0
    for label in ("offered", "at_load"):
        srv = sv.Server(int(200 * (1 << 30)), slots=4, max_batch=8, tiles=tiles)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = srv.run_trace(reqs)
        wall = time.perf_counter() - t0
        rep = sv.trace_report(res, reqs, wall)
        out["traces"].append({"trace": label, "rate_per_s": rate, "p50_s": rep.get("p50_s"), "p99_s": rep.get("p99_s"),
                              "throughput_req_per_s": rep["throughput_req_per_s"], "completed": rep["completed"],
                              "batched_requests": rep["batched_solves"], "wall_s": wall})
        print("serving", json.dumps(out["traces"][-1]), file=sys.stderr, flush=True)
        if label == "offered":
            busy = max(r.finished for r in res.values()) - min(r.admitted for r in res.values())
            capacity = rep["completed"] / busy if busy > 0 else rate
            out["capacity_req_per_s"] = capacity
            rate = load * capacity
            arrivals = sv.poisson_arrivals(n_requests, rate, seed=1)
            reqs = [dataclasses.replace(r, arrival=float(a), ckpt_every=50) for r, a in zip(reqs, arrivals)]
    out["load"] = load
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--members", type=int, default=64)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--horizon", type=int, default=500)
    ap.add_argument("--ckpt-every", type=int, default=0,
                    help="checkpoint interval; 0 = the largest that fits in free HBM (the whole horizon if possible)")
    ap.add_argument("--plain-solves", type=int, default=64,
                    help="one-member solves run one after another (default: the batch's members, equal work)")
    ap.add_argument("--roofline-class", type=int, default=2)
    ap.add_argument("--sample-every", type=int, default=8)
    ap.add_argument("--cpu-steps", type=int, default=150)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph-replays", type=int, default=3,
                    help="also capture the batched solve in a HIP graph and time this many replays (0: skip)")
    for knob in ("row-variant", "row-teams", "adj-variant", "adj-teams", "col-variant", "col-block", "col-split"):
        ap.add_argument("--" + knob, type=int, default=-1, help="FFT tile knob (pa_set_tiles); -1: autotuned")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--ckpt-leg", type=int, default=50,
                    help="also time the solve with checkpoints every this many steps (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=20,
                    help="requests of the short serving trace (0: skip)")
    ap.add_argument("--serving-load", type=float, default=0.8,
                    help="second serving trace at this fraction of the capacity the first one measured")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one torch copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(members and requests would shard across GPUs with no exchange). Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2602_14016_amd import Solver
    from paper_2602_14016_amd.roofline import CLASS_NAMES, HBM_PEAK_GBS, algorithmic_bytes, read_traffic

    N, B, H = args.N, args.members, args.horizon
    nu, dt, k0 = 1e-4, 2e-3, 10.0
    nshell = (N - 1) // 3
    ix = iy = N // 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    from paper_2602_14016_amd.autotune import autotune
    s = Solver(N, B, nu=nu, dt=dt, device=dev)
    w0 = s.init_field(list(range(B)), kind=0, k0=k0, target=0.5)
    torch.cuda.synchronize()
    knobs = ("row_variant", "row_teams", "adj_variant", "adj_teams", "col_variant", "col_block", "col_split")
    manual = any(getattr(args, k) >= 0 for k in knobs)

    def tune(solver, omega0):
        if manual or args.no_autotune:
            solver.set_tiles(**{k: getattr(args, k) for k in knobs})
            return solver.get_tiles() | {"autotuned": False}
        at = autotune(solver, omega0, n_steps=8)
        out = {k: at[k] for k in knobs} | {"autotuned": True}
        out["trials"] = [[r["pass"], r["variant"], r["block"]] + ([r["split"]] if "split" in r else [])
                         + [round(r["ms"], 3)] for r in at["trials"]]
        print("autotune", json.dumps(out), file=sys.stderr, flush=True)
        return out

    tiles = tune(s, w0)

    def ckpt_interval(solver):
        if args.ckpt_every:
            return args.ckpt_every
        torch.cuda.empty_cache()
        k = solver.fit_ckpt_every(H)
        if k < 1:
            print("workload does not fit in device memory", file=sys.stderr)
            sys.exit(1)
        return k

    K = ckpt_interval(s)
    for _ in range(args.warmup):
        s.adjoint_impulse(w0, H, ix, iy, nshell, ckpt_every=K)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    lat = []
    s.profile_start(args.roofline_class, args.sample_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        s.adjoint_impulse(w0, H, ix, iy, nshell, ckpt_every=K)
        e1.record(stream)
        lat.append((e0, e1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = s.profile_stop()
    lat_ms = [a.elapsed_time(b) for a, b in lat]
    elapsed = t1 - t0
    value = B * N * N * H * args.steps / elapsed

    # the same solve captured once into a HIP graph and replayed
    graph = None
    if args.graph_replays:
        from paper_2602_14016_amd.graph import CapturedSolve
        cap = CapturedSolve(lambda: s.adjoint_impulse(w0, H, ix, iy, nshell, ckpt_every=K))
        g0 = torch.cuda.Event(enable_timing=True)
        g1 = torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(args.graph_replays):
            cap.replay()
        g1.record(stream)
        torch.cuda.synchronize()
        gms = g0.elapsed_time(g1) / args.graph_replays
        graph = {"ms_per_step": gms, "replays": args.graph_replays,
                 "grid_point_steps_per_s": B * N * N * H / (gms * 1e-3)}
        del cap

    # the same solve with checkpoints every ckpt_leg steps: forward sweep, segment recomputation, adjoint
    ckpt_leg = None
    if args.ckpt_leg and args.ckpt_leg < H:
        Kc = args.ckpt_leg
        s.adjoint_impulse(w0, H, ix, iy, nshell, ckpt_every=Kc)
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 5))
        c0 = time.perf_counter()
        for _ in range(reps):
            s.adjoint_impulse(w0, H, ix, iy, nshell, ckpt_every=Kc)
        torch.cuda.synchronize()
        cms = 1e3 * (time.perf_counter() - c0) / reps
        ckpt_leg = {"ckpt_every": Kc, "value": B * N * N * H / (cms * 1e-3), "unit": "grid-point-steps/s",
                    "ms_per_step": cms, "steps": reps}

    # plain path: one member per solve, same kernels, solved one after another
    s.close()
    del s
    torch.cuda.empty_cache()
    p = Solver(N, 1, nu=nu, dt=dt, device=dev)
    plain_tiles = None
    if args.plain_solves:
        plain_tiles = tune(p, w0[:1].contiguous())
        plain_tiles.pop("trials", None)
        Kp = ckpt_interval(p)
        plain_tiles["ckpt_every"] = Kp
        p.adjoint_impulse(w0[:1].contiguous(), H, ix, iy, nshell, ckpt_every=Kp)
    torch.cuda.synchronize()
    plain_lat = []
    tp0 = time.perf_counter()
    for m in range(args.plain_solves):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        p.adjoint_impulse(w0[m % B:m % B + 1].contiguous(), H, ix, iy, nshell, ckpt_every=Kp)
        e1.record(stream)
        plain_lat.append((e0, e1))
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    plain_ms = [a.elapsed_time(b) for a, b in plain_lat]
    plain_value = N * N * H * args.plain_solves / (tp1 - tp0) if args.plain_solves else None

    # roofline of the dominant kernel
    cls = args.roofline_class
    per_launch_ms = prof["total_ms"] / max(prof["timed_launches"], 1)
    bytes_launch = algorithmic_bytes(cls, N) * B
    achieved = bytes_launch / (per_launch_ms * 1e-3) / 1e9
    variant = tiles["adj_variant"] if cls >= 2 else tiles["row_variant"] if cls == 0 else tiles["col_variant"]
    kname = CLASS_NAMES[cls].split(" ")[0]
    if cls in (0, 2):
        kname = f"{kname.replace('_kernel', '_pipe_kernel')}<{N}>" if variant == 3 else f"{kname}<{N}, {variant}>"
    else:
        kname = None
    traffic = read_traffic(cls, N, B, kernel=kname)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": CLASS_NAMES[cls], "avg_launch_ms": round(per_launch_ms, 4),
                "algorithmic_bytes_per_launch": int(bytes_launch),
                "timed_launches": prof["timed_launches"], "launches": prof["launches"]}

    p.close()
    del p
    torch.cuda.empty_cache()
    serving = None
    if args.serving_requests:
        serving = serving_leg(args.serving_requests, args.serving_load, dev)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(N, nu, dt, args.cpu_steps, k0)

    line = {
        "metric": METRIC, "value": value, "unit": "grid-point-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ensemble of {B} realizations of {N}^2 decaying 2D turbulence "
                               f"(k0={k0:g} random-phase spectrum, energy 0.5, seeds 0..{B - 1}), nu={nu:g}, "
                               f"dt={dt:g}, {H} forward + {H} adjoint steps per member from a unit u-impulse "
                               f"at ({ix},{iy}), "
                               + (f"checkpoints every {K}" if K < H else "whole stage trajectory kept in HBM (no recomputation)")
                               + f", shell energies |k|=1..{nshell}",
                   "members": B, "grid": N, "horizon": H, "ckpt_every": K},
        "latency_ms": {"batched_p50": percentile(lat_ms, 50), "batched_p99": percentile(lat_ms, 99),
                       "plain_p50": percentile(plain_ms, 50), "plain_p99": percentile(plain_ms, 99)},
        "plain": {"value": plain_value, "unit": "grid-point-steps/s", "solves": args.plain_solves, "tiles": plain_tiles,
                  "speedup_batched_over_plain": value / plain_value if plain_value else None},
        "roofline": roofline,
        "graph": graph,
        "checkpointed": ckpt_leg,
        "serving": serving,
        "tiles": tiles,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
