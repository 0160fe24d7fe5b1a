"""Build the HIP library libpadjoint.so in-tree for gfx950.

    python -m paper_2602_14016_amd.build          (or build() from Python)

Every .hip file under csrc/ is compiled with hipcc for the CDNA4 target and
linked into one shared library next to this file.  Packed FP32 instructions
are disabled for all device code (the build never relies on them).
"""

import os
import shlex
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpadjoint.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PA_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# -ffp-contract=on: a multiply is fused into an add only within one source
# expression, decided in the front end, so every copy of a piece of code
# (a peeled loop iteration, a kernel variant) rounds identically; with "fast"
# the backend fuses across statements where it finds the pattern, and two
# copies of the same source can differ in the last bit.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable", "-ffp-contract=on"]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _run(cmd):
    t0 = time.time()
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("command failed: " + " ".join(shlex.quote(c) for c in cmd))
    return time.time() - t0, r.stdout


def build(verbose=True, jobs=None):
    """Compile every source and link libpadjoint.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if jobs is None:
        jobs = max(1, min(8, os.cpu_count() or 1))
    objs = []
    procs = []
    for src in sources():
        obj = os.path.join(BUILD_DIR, os.path.basename(src)[:-4] + ".o")
        cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-c", src, "-o", obj]
        procs.append((src, obj, cmd))
    # compile in parallel
    running = []
    t0 = time.time()
    for src, obj, cmd in procs:
        while len(running) >= jobs:
            _wait_one(running)
        running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    while running:
        _wait_one(running)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s")
    return LIB


def _wait_one(running):
    src, p = running.pop(0)
    out, _ = p.communicate()
    if p.returncode != 0:
        sys.stderr.write(out)
        raise RuntimeError(f"hipcc failed on {src}")
    if out.strip():
        # keep warnings visible but short
        lines = [l for l in out.splitlines() if "warning" in l and "packed-fp32" not in l]
        for l in lines[:20]:
            print(l)


if __name__ == "__main__":
    build()
