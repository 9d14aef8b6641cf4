"""Host-side schedule of the H-Cholesky, checked under AddressSanitizer and
UndefinedBehaviorSanitizer.

tests/host/plan_check.cpp builds the cluster tree, block tree and plan of the
library's own host code (tree.cpp) for 53 point sets (uniform 2-D and 3-D at
ragged sizes from 1 to 20,000, leaf sizes 1 to 128, collinear, duplicated and all-equal points,
batches of 5 and 64 problems, eta from 0.5 to 4) and checks invariants that
follow from the left-looking block Cholesky on a partition of the lower
triangle (Section 2): the blocks tile each problem's lower triangle once, each
entry's external update pairs cover exactly the columns to its left, the
chunk, Gram, column-solve and inner-update lists cover their work once and in
an order where every input is final before it is read, and the low-rank
targets' sketch lists (pieces, chunks, input-side products and their segments,
row tiles) cover their terms once. Seven smaller configurations (2-D, 3-D, a
batch of three, eta 0.01, 4 and 50, leaf size 1) are then executed in exact dense
arithmetic in the order of the plan's steps; the factor must equal a textbook
Cholesky factor of the same matrix to 1e-11 relative, and the forward
substitution by the plan's solve lists, and the backward one by the same lists
in reverse (the kriging solve), textbook substitutions to 1e-10; the sampler's
product L w by row panels equals the plain product. Then 200 random
configurations (fixed seed: dimension, problems per batch, point layouts with
duplicates, collinear or anisotropic points, leaf size, eta, storage width and
schedule options) go through the same invariants, the small ones also through
the exact execution. No GPU is used; the
program is compiled with g++ against the host half of the HIP headers.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"


def test_plan_invariants_sanitized(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path / "plan_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE,
           os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           os.path.join(ROOT, "paper_2104_07146_amd", "csrc", "tree.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(run.stdout[-3000:])
    assert run.returncode == 0, (run.stdout[-3000:], run.stderr[-4000:])
    lines = run.stdout.splitlines()
    assert sum(l.startswith("ok ") and not l.startswith("ok random") for l in lines) == 53
    assert sum(l.startswith("ok random") for l in lines) == 200
    assert sum(l.startswith("exact ") and not l.startswith("exact random") for l in lines) == 7
    assert sum(l.startswith("exact random") for l in lines) >= 5
    assert "runtime error" not in run.stderr
