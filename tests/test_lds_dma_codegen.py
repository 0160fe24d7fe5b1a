"""Code-generation check of the pipelined row kernels' global->LDS loads (CPU; needs hipcc).

A global->LDS load takes its LDS base from M0, which must be uniform over
the wavefront; the compiler sets it with v_readfirstlane.  If the compiler
merged a masked load with a load of another LDS base, the VGPR feeding M0
would carry two values (one per lane subset) and every lane would take one
lane's base.  For every such load in the generated gfx950 assembly, the VGPR
feeding M0 must have a single definition in the kernel or be (re)defined in
the load's own basic block.
"""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_14016_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def m0_problems(asm):
    problems = []
    for name in [x for x in re.findall(r"^(_ZN2pa\S+):", asm, re.M) if "pipe" in x]:
        st = asm.index(name + ":")
        en = asm.index(".Lfunc_end", st)
        lines = [l.strip() for l in asm[st:en].splitlines() if l.strip() and not l.strip().startswith(";")]
        block_start = 0
        for i, l in enumerate(lines):
            if l.endswith(":"):
                block_start = i
            if "global_load_lds" not in l:
                continue
            j = i - 1
            while j > block_start and not re.match(r"s_mov_b32 m0, (s\d+)", lines[j]):
                j -= 1
            m = re.match(r"s_mov_b32 m0, (s\d+)", lines[j])
            if not m:
                problems.append((name, i, "no M0 write in the load's block"))
                continue
            sreg = m.group(1)
            k = j - 1
            while k > block_start and not re.match(rf"v_readfirstlane_b32 {sreg}, (v\d+)", lines[k]):
                k -= 1
            r = re.match(rf"v_readfirstlane_b32 {sreg}, (v\d+)", lines[k])
            if not r:
                problems.append((name, i, "M0 not set from a readfirstlane in the load's block"))
                continue
            vreg = r.group(1)
            defs = [q for q, x in enumerate(lines)
                    if re.match(rf"v_\w+ {vreg},", x) or re.match(rf"v_\w+ v\[{vreg[1:]}:", x)]
            if not any(block_start < q < k for q in defs) and len(defs) != 1:
                problems.append((name, i, f"{vreg} has {len(defs)} definitions, none in the load's block"))
    return problems


def test_checker_flags_a_merged_load():
    # two definitions of the M0 source reaching a load after a join
    asm = """_ZN2pa19row_adj_pipe_kernelILi8EEEvNS_4DimsENS_7RowArgsEi:
\tv_add_u32_e32 v10, 0xa00, v139
\ts_and_saveexec_b64 s[0:1], vcc
\tv_add_u32_e32 v10, 0x600, v139
.LBB0_1:
\ts_or_b64 exec, exec, s[0:1]
\tv_readfirstlane_b32 s0, v10
\ts_mov_b32 m0, s0
\tglobal_load_lds_dwordx4 v[4:5], off
.Lfunc_end0:
"""
    assert len(m0_problems(asm)) == 1


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
@pytest.mark.parametrize("N", [64, 256])
def test_pipelined_loads_take_a_uniform_lds_base(N, tmp_path):
    out = tmp_path / f"k{N}.s"
    cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-ffp-contract=on", "--offload-device-only", "-S",
           os.path.join(CSRC, f"kern_{N}.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    asm = out.read_text()
    assert asm.count("global_load_lds_dwordx4") > 0
    assert m0_problems(asm) == []
