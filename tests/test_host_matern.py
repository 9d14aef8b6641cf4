"""The library's Matern evaluation (csrc/matern.hpp with the parameter setup
of csrc/common.hpp), compiled for the host, against the oracle's Matern
(SciPy's exponentially scaled K_nu) over the whole smoothness range the
library accepts, nu in [0.05, 8], and distances from 1e-8 to the cut-off.

The GPU parity test checks the device build at a few nu; this test sweeps
170 values of nu, including the closed-form orders 1/2, 3/2, 5/2 and their
neighbours, where the general path takes over, at 150 distances each.
Bars: float64 within 1.5e-13 + 4e-16 x relative wherever the value exceeds
1e-290 (the second term is the conditioning of exp(-x) to the rounding of
x = h / ell, which the oracle does not share: about x times the unit
roundoff); float32
within 1e-5 relative where the value exceeds 1e-30 below its cut-off
(x <= 100), the approximation accuracy the mixed path is used with (values
never exceed sigma^2, so this also bounds the absolute error by 1e-5 sigma^2).
No GPU is used.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import matern

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path_factory.mktemp("matern") / "matern_check")
    cmd = [gxx, "-std=c++17", "-O2", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE, os.path.join(ROOT, "tests", "host", "matern_check.cpp"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    return exe


def _eval(exe, rows):
    text = "\n".join(" ".join(repr(float(v)) for v in r) for r in rows)
    r = subprocess.run([exe], input=text, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-3000:]
    vals = np.array([[float(v) for v in line.split()] for line in r.stdout.splitlines()])
    return vals[:, 0], vals[:, 1]


def test_matern_whole_nu_range(driver):
    nus = np.concatenate([np.linspace(0.05, 8.0, 160),
                          [0.5, 1.5, 2.5, 0.4999999, 0.5000001, 1.4999999, 2.5000001, 1.0, 2.0, 7.9999]])
    x = np.concatenate([np.geomspace(1e-8, 1, 40), np.linspace(1.0, 40, 80), np.geomspace(40, 700, 30)])
    sigma2, ell = 1.7, 0.13
    rows = [(sigma2, ell, nu, xi * ell) for nu in nus for xi in x]
    got64, got32 = _eval(driver, rows)
    got64 = got64.reshape(len(nus), len(x))
    got32 = got32.reshape(len(nus), len(x))
    worst64 = worst32 = worst_abs = 0.0
    for i, nu in enumerate(nus):
        want = matern.matern(x * ell, sigma2, ell, nu)
        big = want > 1e-290
        e64 = np.abs(got64[i][big] - want[big]) / want[big]
        bar = 1.5e-13 + 4e-16 * x[big]
        assert np.all(e64 <= bar), (nu, float(np.max(e64 / bar)), x[big][np.argmax(e64 / bar)])
        sel = (want > 1e-30) & (x <= 100)
        e32 = np.abs(got32[i][sel] - want[sel]) / want[sel]
        assert e32.max() <= 1e-5, (nu, float(e32.max()), x[sel][np.argmax(e32)])
        ea = np.abs(got32[i][x <= 100] - want[x <= 100]) / sigma2
        worst64, worst32, worst_abs = max(worst64, e64.max()), max(worst32, e32.max()), max(worst_abs, ea.max())
    print(f"float64 worst relative {worst64:.3e}; float32 worst relative {worst32:.3e}, "
          f"worst absolute / sigma2 {worst_abs:.3e}")


def test_matern_limits_and_closed_forms(driver):
    sigma2, ell = 2.0, 0.5
    rows = [(sigma2, ell, nu, 0.0) for nu in (0.05, 0.5, 1.3, 8.0)]
    rows += [(sigma2, ell, 0.5, 0.3), (sigma2, ell, 1.5, 0.3), (sigma2, ell, 2.5, 0.3)]
    rows += [(sigma2, ell, 1.3, 800.0 * ell)]
    v64, v32 = _eval(driver, rows)
    assert np.all(v64[:4] == sigma2) and np.all(v32[:4] == np.float32(sigma2))   # M(0) = sigma^2
    x = 0.3 / ell
    closed = sigma2 * np.exp(-x) * np.array([1.0, 1.0 + x, 1.0 + x + x * x / 3.0])
    assert np.allclose(v64[4:7], closed, rtol=1e-15, atol=0)
    assert v64[7] == 0.0 and v32[7] == 0.0     # beyond the cut-off
