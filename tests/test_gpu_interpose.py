"""The HIP API interposer end to end: the paper's example program (Sec. 4,
Listing 2) run under LD_PRELOAD prints the report of Listing 6 and its copy
is refused; the corrected program runs clean.  The program is built with the
library (build()) and started as a child process."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PRELOAD = os.path.join(ROOT, "paper_1310_0901_amd", "libxfercheck_preload.so")
EXAMPLE = os.path.join(ROOT, "tests", "native", "worked_example")


def run_example(arg):
    env = dict(os.environ)
    env["LD_PRELOAD"] = (env["LD_PRELOAD"] + ":" if env.get("LD_PRELOAD") else "") + PRELOAD
    env["XC_POOL_BYTES"] = str(64 << 20)
    print(f"[interpose] running worked_example {arg}", flush=True)
    return subprocess.run([EXAMPLE, arg], env=env, capture_output=True, text=True, timeout=120)


def test_worked_example_report():
    assert os.path.exists(PRELOAD) and os.path.exists(EXAMPLE), "build() first"
    fx = json.load(open(os.path.join(ROOT, "tests", "golden", "pin1_worked_example.json")))
    r = run_example("faulty")
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    lines = r.stderr.splitlines()
    i = lines.index(fx["report_lines"][0])
    assert lines[i + 1] == fx["report_lines"][1]
    assert "hipMemcpyDeviceToHost" in lines[i + 2]
    assert "hipMemcpy returned 1 " in r.stdout          # hipErrorInvalidValue: the copy was refused
    assert "1 copies checked, 1 with errors" in r.stderr


def test_corrected_program_is_clean():
    r = run_example("correct")
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    assert "Error" not in r.stderr
    assert "hipMemcpy returned 0 " in r.stdout
    assert "1 copies checked, 0 with errors" in r.stderr
