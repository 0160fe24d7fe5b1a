"""bench.py's command-line contract on the CPU: one GPU only (--gpus N > 1, or a
multi-rank launch, exits with a message before touching a device), and the
JSON line it prints carries the contract's keys (checked on the source of the
line, since printing it needs the device)."""

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def _run(args, env=None):
    e = dict(os.environ)
    e.update(env or {})
    return subprocess.run([sys.executable, BENCH] + args, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                          text=True, env=e, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    for args, env in ((["--gpus", "2"], None), (["--gpus", "8"], None), ([], {"WORLD_SIZE": "2"})):
        r = _run(args, env)
        assert r.returncode == 2, (args, r.returncode, r.stderr)
        assert "one GPU only" in r.stderr and r.stdout == ""


def test_result_line_has_the_contract_keys():
    src = open(BENCH).read()
    line = src[src.index("line = {"):src.index("print(json.dumps(line)")]
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "checkpointed",
                "serving"):
        assert re.search(r'"%s"\s*:' % key, line), key
    roof = src[src.index("roofline = {"):src.index("cpu = None")]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert re.search(r'"%s"\s*:' % key, roof), key
