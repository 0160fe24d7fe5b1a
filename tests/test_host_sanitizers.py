"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

api.hip is compiled with both sanitizers on its host code only (every
-fsanitize flag goes to the host pass; the device code is built as usual) and
linked, with the library's other objects as built, into abi_host_driver.cpp.
The C++ program calls the entry points that run without a device: argument
validation before any device call, and the binomial checkpoint schedule over
every chain of up to 80 segments under budgets 1..10 plus long chains, each
schedule replayed and its advance count compared with the optimum.  Any
sanitizer report fails the test.
"""

import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_14016_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2602_14016_amd", "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _objects():
    objs = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))] if os.path.isdir(BUILD) else []
    objs = [o for o in objs if o.endswith(".o") and os.path.basename(o) != "api.o"]
    if not objs:
        from paper_2602_14016_amd import build
        build.build(verbose=False)
        objs = [os.path.join(BUILD, f) for f in sorted(os.listdir(BUILD))
                if f.endswith(".o") and f != "api.o"]
    return objs


def _run(cmd, **kw):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-4000:]
    return r.stdout


@pytest.mark.timeout(600)
def test_abi_host_code_is_clean_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    from paper_2602_14016_amd.build import ARCH, COMMON, DEVICE_FLAGS
    api_o = str(tmp_path / "api_san.o")
    drv_o = str(tmp_path / "driver.o")
    exe = str(tmp_path / "abi_host_driver")
    flags = [f for f in COMMON if f != "-O3"] + ["-O1", "-g"]
    _run([HIPCC] + flags + DEVICE_FLAGS + HOST_SAN + ["-c", os.path.join(CSRC, "api.hip"), "-o", api_o])
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include")] + HOST_SAN +
         ["-c", os.path.join(ROOT, "tests", "abi_host_driver.cpp"), "-o", drv_o])
    _run([HIPCC, f"--offload-arch={ARCH}"] + HOST_SAN + [drv_o, api_o] + _objects() + ["-o", exe])
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_leaks=1:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env, timeout=300)
    out = r.stdout
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert out.strip().splitlines()[-1] == "ok"
