"""Build the HIP library libhmle.so in-tree for gfx950 (hipcc). The oracle is
plain Python (NumPy / SciPy) and needs no build. Run:
python -m paper_2104_07146_amd.build"""
from __future__ import annotations

import os
import shlex
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libhmle.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-variable", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [
    ("kernels.hip", ["-x", "hip"]),
    ("learned.hip", ["-x", "hip"]),
    ("tree_gpu.hip", ["-x", "hip", "-ffp-contract=off"]),
    ("learned_api.cpp", []),
    ("api.cpp", []),
    ("fit.cpp", []),
    ("tree.cpp", ["-ffp-contract=off"]),
]


def _run(cmd):
    print("+", " ".join(shlex.quote(c) for c in cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    for src, extra in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        _run([HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
