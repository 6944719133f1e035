"""Build the transfer checker's native libraries in-tree.

    python -m paper_1310_0901_amd.build

compiles csrc/*.hip and csrc/*.cpp for gfx950 into
paper_1310_0901_amd/libxfercheck.so (hipcc), and, for the host-side CPU
tests, csrc/host_logic.cpp into a standalone sanitizer test binary.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libxfercheck.so")
PRELOAD = os.path.join(HERE, "libxfercheck_preload.so")
EXAMPLE_SRC = os.path.join(ROOT, "tests", "native", "worked_example.hip")
EXAMPLE = os.path.join(ROOT, "tests", "native", "worked_example")
ARCH = os.environ.get("XC_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function", f"-I{os.path.join(ROOT, 'include')}"]
SOURCES = ["kernels.hip", "table.hip", "sort.hip", "segment.hip", "shadowindex.hip", "race.hip", "strided.hip", "runtime.cpp",
           "host_logic.cpp", "format.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        _run(["hipcc", *HIP_FLAGS, *lang, "-c", path, "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run(["hipcc", "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # the HIP API interposer (LD_PRELOAD), linked against the library
    tmp = PRELOAD + ".tmp"
    _run(["hipcc", *HIP_FLAGS, "-x", "hip", "-shared", "-o", tmp, os.path.join(CSRC, "interpose.cpp"),
          f"-L{HERE}", "-lxfercheck", "-Wl,-rpath,$ORIGIN", "-ldl"])
    os.replace(tmp, PRELOAD)
    # the paper's example program, run under the interposer by the tests
    _run(["hipcc", "-O2", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-o", EXAMPLE, EXAMPLE_SRC])
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
