"""Algorithmic byte model of the hot kernels and the HBM-traffic record.

Kernel classes are those the library's launch timer knows (pa_profile_start):
0 the right-hand-side row pass, 1 the forward-stage column pass, 2 the
adjoint-product row pass, 3 the adjoint-stage column pass.

Algorithmic bytes count what a kernel must move per member and launch, with
every field read or written once: Yb is one field in the Y layout restricted
to the retained band, N rows of Kc + 1 complex values; Cb is one compact
spectral state, (2 Kc + 1) x (Kc + 1) complex values.  Padding columns and
repeated reads are not counted, so achieved = algorithmic bytes / time is a
lower bound on the bandwidth a kernel actually draws.
"""

import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E

CLASS_NAMES = {0: "row_nl_kernel", 1: "col_kernel (forward stages)", 2: "row_adj_kernel",
               3: "col_kernel (adjoint stages)"}


def field_bytes(N):
    """(Yb, Cb) for grid size N."""
    Kc = (N - 1) // 3
    return N * (Kc + 1) * 16, (2 * Kc + 1) * (Kc + 1) * 16


def algorithmic_bytes(cls, N):
    """Bytes per member of one launch of kernel class cls."""
    Yb, Cb = field_bytes(N)
    return {0: 5 * Yb,                  # read U, V, Wx, Wy; write q
            1: 5 * Yb + 2.75 * Cb,      # read q; write U, V, Wx, Wy; state and accumulator (mean over stages A-D)
            2: 8 * Yb,                  # read U, V, Wx, Wy, Lambda, Lambda_y; write the two products
            3: 4 * Yb + 2.5 * Cb}[cls]  # read the two products; write Lambda, Lambda_y; adjoint accumulators


# per column-pass mode (col_kernel<N, V, MODE>): bytes per member
def column_mode_bytes(mode, N):
    Yb, Cb = field_bytes(N)
    return {1: 5 * Yb + 2 * Cb,    # stage A: read q, omega; write acc, 4 fields
            2: 5 * Yb + 3 * Cb,    # stage B: read q, omega, acc; write acc, 4 fields
            3: 5 * Yb + 3 * Cb,    # stage C
            4: 5 * Yb + 3 * Cb,    # stage D: read q, omega, acc; write omega, 4 fields
            7: 4 * Yb + 2 * Cb,    # adjoint C: read 2 products, lambda; write omega-bar, 2 fields
            8: 4 * Yb + 3 * Cb,    # adjoint B: read 2 products, lambda, omega-bar; write omega-bar, 2 fields
            9: 4 * Yb + 3 * Cb,    # adjoint A
            10: 4 * Yb + 2 * Cb}.get(mode)  # adjoint n: read 2 products, omega-bar; write lambda, 2 fields


# the sources that define and instantiate the row and column kernels, and the
# build flags they are compiled with (host-side files do not change them)
KERNEL_SOURCES = ("csrc/fft.hpp", "csrc/kernels.hpp", "csrc/kernels_impl.hpp", "csrc/kernels.hip",
                  "csrc/kern_8.hip", "csrc/kern_16.hip", "csrc/kern_32.hip", "csrc/kern_64.hip",
                  "csrc/kern_128.hip", "csrc/kern_256.hip", "csrc/kern_512.hip", "csrc/kern_1024.hip", "build.py")


def kernel_source_sha():
    """Hash of the row/column kernel sources and build flags: a traffic record
    applies only to the kernels it was taken on."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic_counters.txt")


def read_traffic(cls, N, members, kernel=None, path=TRAFFIC_PATH):
    """HBM bytes per launch of class cls from the committed counter record, or
    None if the record is missing or was taken on other sources, another
    class, shape or (if given) another kernel instantiation."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha") != kernel_source_sha():
        return None
    try:
        if int(kv.get("class", -1)) != cls or int(kv.get("N", -1)) != N or int(kv.get("members", -1)) != members:
            return None
        if kernel is not None and kv.get("kernel") != kernel:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
