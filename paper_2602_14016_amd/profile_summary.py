"""Turn rocprofv3 CSV output into the short text summaries kept in profiles/.

    python -m paper_2602_14016_amd.profile_summary stats KERNEL_STATS_CSV --command CMD --title T --out FILE
    python -m paper_2602_14016_amd.profile_summary traffic FETCH_CSV WRITE_CSV --command CMD --members B --N N \
        --cls C --kernel NAME --calib-mib M --out FILE
    python -m paper_2602_14016_amd.profile_summary counters CSV [CSV ...] --command CMD --title T \
        --kernels NAME [NAME ...] --out FILE

stats: per-kernel calls, average and total duration from a --kernel-trace
--stats run (run_kernel_stats.csv).

traffic: per-kernel HBM bytes per dispatch from two --pmc runs
(run_counter_collection.csv of FETCH_SIZE and of WRITE_SIZE, KiB per
dispatch).  Each counter is scaled by what it reads for a device copy of
known size in the same run (the largest __amd_rocclr_copyBuffer dispatch of a
--calib-copy-mib copy), then set beside the algorithmic read and write bytes
of the kernel (roofline.py).  The record for kernel NAME of class C is what
bench.py reports as roofline.traffic while the sources are unchanged.
"""

import argparse
import collections
import csv
import re
import sys

from .roofline import field_bytes, kernel_source_sha


def kernel_rw_bytes(name, N):
    """Algorithmic (read, write) bytes per member of one dispatch of kernel `name`, or None."""
    Yb, Cb = field_bytes(N)
    if name.startswith("row_nl"):
        return 4 * Yb, Yb
    if name.startswith("row_adj"):
        return 6 * Yb, 2 * Yb
    m = re.match(r"col_kernel<\d+, \d+, (\d+)>", name)
    if not m:
        return None
    mode = int(m.group(1))
    return {1: (Yb + Cb, 4 * Yb + Cb), 2: (Yb + 2 * Cb, 4 * Yb + Cb), 3: (Yb + 2 * Cb, 4 * Yb + Cb),
            4: (Yb + 2 * Cb, 4 * Yb + Cb), 7: (2 * Yb + Cb, 2 * Yb + Cb), 8: (2 * Yb + 2 * Cb, 2 * Yb + Cb),
            9: (2 * Yb + 2 * Cb, 2 * Yb + Cb), 10: (2 * Yb + Cb, 2 * Yb + Cb)}.get(mode)


def short(name):
    return name.split("(")[0].replace("void ", "").replace("pa::", "").strip()


def stats(args):
    rows = list(csv.DictReader(open(args.csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# {args.title}", "#", "# command (from /tmp, TMPDIR=/tmp; REPO = repository root):"]
    out += [f"#   {line}" for line in args.command.split("\n")]
    out += ["#", f"# {'kernel':44s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>10s} {'share':>6s}"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[: args.top]:
        out.append(f"  {short(r['Name'])[:44]:44s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:9.2f} "
                   f"{float(r['TotalDurationNs']) / 1e6:10.2f} {100 * float(r['TotalDurationNs']) / tot:5.1f}%")
    out.append(f"# total kernel time {tot / 1e6:.2f} ms over {sum(int(r['Calls']) for r in rows)} dispatches")
    return "\n".join(out) + "\n"


def per_kernel_kib(path, counter):
    vals = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            vals[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def traffic(args):
    fetch = per_kernel_kib(args.fetch_csv, "FETCH_SIZE")
    write = per_kernel_kib(args.write_csv, "WRITE_SIZE")
    calib = args.calib_mib * (1 << 20)
    cf = max(fetch.get("__amd_rocclr_copyBuffer", [0.0]))
    cw = max(write.get("__amd_rocclr_copyBuffer", [0.0]))
    if cf <= 0 or cw <= 0:
        raise SystemExit("no calibration copy dispatch found")
    sf, sw = calib / (cf * 1024), calib / (cw * 1024)
    out = [f"# HBM traffic per launch from rocprofv3 counters (KiB per dispatch), B = {args.members}, N = {args.N}",
           "#", "# commands (from /tmp, TMPDIR=/tmp; REPO = repository root), one pass per counter:"]
    out += [f"#   {line}" for line in args.command.split("\n")]
    out += ["# calibration: the device copy of --calib-copy-mib MiB (__amd_rocclr_copyBuffer, largest dispatch)",
            "#   in the same run; scale = true bytes / counter bytes, applied to every kernel's counter", "#",
            f"calib_copy_bytes: {calib}", f"calib_fetch_kib: {cf:.2f}", f"calib_write_kib: {cw:.2f}",
            f"scale_fetch: {sf:.4f}", f"scale_write: {sw:.4f}", "#",
            f"# {'kernel':34s} {'read_MB':>9s} {'alg_read_MB':>12s} {'write_MB':>9s} {'alg_write_MB':>13s}"]
    for k in sorted(set(fetch) & set(write)):
        rw = kernel_rw_bytes(k, args.N)
        if rw is None:
            continue
        rd = sf * 1024 * sum(fetch[k]) / len(fetch[k]) / 1e6
        wr = sw * 1024 * sum(write[k]) / len(write[k]) / 1e6
        out.append(f"# {k[:34]:34s} {rd:9.2f} {rw[0] * args.members / 1e6:12.2f} {wr:9.2f} "
                   f"{rw[1] * args.members / 1e6:13.2f}")
    if args.kernel not in fetch or args.kernel not in write:
        raise SystemExit(f"kernel {args.kernel!r} not in the counter runs: {sorted(fetch)}")
    fk = sum(fetch[args.kernel]) / len(fetch[args.kernel])
    wk = sum(write[args.kernel]) / len(write[args.kernel])
    out += ["#", "# dominant kernel used by bench.py's roofline 'traffic':", f"class: {args.cls}", f"N: {args.N}",
            f"members: {args.members}", f"kernel: {args.kernel}", f"fetch_kib_per_launch: {fk:.2f}",
            f"write_kib_per_launch: {wk:.2f}", f"hbm_bytes_per_launch: {int(round(1024 * (sf * fk + sw * wk)))}",
            f"source_sha: {kernel_source_sha()}"]
    return "\n".join(out) + "\n"


def counters(args):
    """Mean per dispatch of every counter in the --pmc runs, for the named kernels,
    with the wave-cycle shares of the SQ wait and issue counters."""
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in args.csv:
        for r in csv.DictReader(open(path)):
            vals[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = [f"# {args.title}", "#", "# commands (from /tmp, TMPDIR=/tmp; REPO = repository root), one pass each:"]
    out += [f"#   {line}" for line in args.command.split("\n")]
    out += ["#", "# mean per dispatch; shares are of SQ_WAVE_CYCLES (summed wave residency)", f"source_sha: {kernel_source_sha()}"]
    for k in args.kernels:
        if k not in vals:
            raise SystemExit(f"kernel {k!r} not in the counter runs: {sorted(vals)}")
        d = {c: sum(v) / len(v) for c, v in vals[k].items()}
        out += ["", f"kernel: {k}"]
        for c in sorted(d):
            out.append(f"  {c:28s} {d[c]:16.6g}")
        wc = d.get("SQ_WAVE_CYCLES")
        if wc:
            for c in ("SQ_ACTIVE_INST_VALU", "SQ_WAIT_INST_LDS", "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_LDS"):
                if c in d:
                    out.append(f"  share {c:22s} {d[c] / wc:8.3f}")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--command", required=True)
    a.add_argument("--title", required=True)
    a.add_argument("--top", type=int, default=20)
    a.add_argument("--out", required=True)
    b = sub.add_parser("traffic")
    b.add_argument("fetch_csv")
    b.add_argument("write_csv")
    b.add_argument("--command", required=True)
    b.add_argument("--members", type=int, required=True)
    b.add_argument("--N", type=int, required=True)
    b.add_argument("--cls", type=int, required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--calib-mib", type=int, required=True)
    b.add_argument("--out", required=True)
    c = sub.add_parser("counters")
    c.add_argument("csv", nargs="+")
    c.add_argument("--command", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    text = {"stats": stats, "traffic": traffic, "counters": counters}[args.what](args)
    with open(args.out, "w") as fh:
        fh.write(text)
    sys.stdout.write(text)


if __name__ == "__main__":
    main()
