"""The optimiser of hmle_fit (csrc/fit.cpp: Nelder-Mead in the coordinates of
Section 5.1, optionally with the variance profiled out) checked on the CPU
against SciPy's Nelder-Mead, point by point.

tests/host/fit_core_check.cpp links fit.cpp with a test double of the
evaluation entry points (assemble, factor, loglik) whose log-likelihood is a
smooth analytic function of log(theta) and whose factorisation fails below a
nugget floor; the double prints every point it evaluates. The same search is
run here with scipy.optimize.minimize(method="Nelder-Mead") from the same
initial simplex (x0 and x0 + step e_i in the searched coordinates), the same
objective and the start back-off of hmle_fit (the nugget coordinate lowered by
one until the start evaluates; points outside the parameter box count as
failed evaluations). Every evaluated theta, the evaluation and
iteration counts, the estimate and the log-likelihood must agree: SciPy forms
its centroid and trial points with a different rounding order, hence a
tolerance of 1e-9 in the coordinates instead of bit equality. Compiled with
AddressSanitizer and UndefinedBehaviorSanitizer; no GPU is used.
"""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import optimize

from oracle import reparam

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"
N = 1000.0
CENTRE = (math.log(1.3), math.log(0.12), math.log(0.7), math.log(0.02))
A = ((4, 1, 0.5, 0), (1, 3, 0.8, 0.2), (0.5, 0.8, 2, 0.1), (0, 0.2, 0.1, 1))
B = ((2, 0.3, 0.1), (0.3, 1, 0.2), (0.1, 0.2, 0.5))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(HIP_INCLUDE, "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are not available")
    exe = str(tmp_path_factory.mktemp("fit") / "fit_core_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-D__HIP_PLATFORM_AMD__", "-I" + HIP_INCLUDE,
           os.path.join(ROOT, "tests", "host", "fit_core_check.cpp"),
           os.path.join(ROOT, "paper_2104_07146_amd", "csrc", "fit.cpp"), "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-4000:]
    return exe


def _run(exe, profile, start, step, tol, max_iter, floor, band=0.0):
    s = start if start is not None else (0, 0, 0, 0)
    args = [exe, str(int(profile))] + [repr(float(v)) for v in s] + [repr(step), repr(tol), str(max_iter), repr(floor),
                                                                     repr(band)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr
    evals, result = [], None
    for line in r.stdout.splitlines():
        f = line.split()
        if f[0] == "eval":
            evals.append(tuple(float(v) for v in f[1:]))
        elif f[0] == "result":
            result = dict(status=int(f[1]), theta=tuple(float(v) for v in f[2:6]), evals=int(f[6]),
                          iters=int(f[7]), failed=int(f[8]), converged=int(f[9]), logL=float(f[10]))
    return evals, result


def _full_loglik(t):
    u = [math.log(t[0]) - CENTRE[0], math.log(t[1]) - CENTRE[1], math.log(t[2]) - CENTRE[2],
         math.log(t[3]) - CENTRE[3]]
    q = sum(u[i] * A[i][j] * u[j] for i in range(4) for j in range(4))
    return -(0.5 * q + u[0] ** 4 / 20.0)


def _profile_parts(t):
    v = [math.log(t[1]) - CENTRE[1], math.log(t[2]) - CENTRE[2], math.log(t[3]) - CENTRE[3]]
    q = sum(v[i] * B[i][j] * v[j] for i in range(3) for j in range(3))
    return 10.0 + 50.0 * q, 0.1 * (v[0] ** 2 + v[0] * v[2] + 0.5 * v[2] ** 2) + 0.05 * v[1] ** 2 + 0.01 * v[0]


def _in_box(t):
    """hmle_fit's parameter box (documented with hmle_fit in include/hmle.h)."""
    s2, ell, nu, t2 = t
    return 1e-6 <= s2 <= 1e6 and 1e-4 <= ell <= 10.0 and 0.05 <= nu <= 8.0 and 0.0 <= t2 <= 1e3


def _scipy_search(profile, start, step, tol, max_iter, floor, band=0.0):
    """The search hmle_fit performs, written with SciPy's Nelder-Mead: -logL
    (or the profile value -Lp of eq. (1) at sigma^2 = q / n) over the
    Section 5.1 coordinates."""
    log = []
    calls = [0]

    def point(x):
        t = reparam.to_theta(x)
        return (1.0, t[1], t[2], t[3]) if profile else t

    def value(x, record=True):
        calls[0] += 1
        t = point(x)
        if not _in_box(t):
            return math.inf
        if t[3] < floor or (band > 0 and band <= t[1] < 1.15 * band):
            return math.inf
        if record:
            log.append(t)
        if not profile:
            return -_full_loglik(t)
        h1, h2 = _profile_parts(t)
        q = N * math.exp(h2)
        return 0.5 * N * math.log(2 * math.pi) + 0.5 * h1 + 0.5 * N * math.log(q / N) + 0.5 * N

    x0 = list(reparam.PAPER_START if start is None else reparam.from_theta(start))
    if profile:
        s2, _, _, t2 = reparam.to_theta(x0)
        x0[0] = 0.0
        x0[3] = -math.log(math.sqrt(t2 / s2)) / math.log(2.0)
    f0 = value(x0)
    for _ in range(30):
        if math.isfinite(f0):
            break
        x0[3] -= 1.0
        f0 = value(x0)
    pre_calls = calls[0]
    searched = [1, 2, 3] if profile else [0, 1, 2, 3]
    y0 = np.array([x0[d] for d in searched])
    simplex = np.array([y0] + [y0 + step * np.eye(len(y0))[i] for i in range(len(y0))])
    first = [True]

    def fun(y):
        x = list(x0)
        for k, d in enumerate(searched):
            x[d] = float(y[k])
        if first[0]:       # the start itself, already evaluated above
            first[0] = False
            return f0
        return value(x)

    res = optimize.minimize(fun, y0, method="Nelder-Mead",
                            options={"initial_simplex": simplex, "xatol": tol, "fatol": np.inf,
                                     "maxiter": max_iter + 1, "maxfev": 10 ** 9})
    x = list(x0)
    for k, d in enumerate(searched):
        x[d] = float(res.x[k])
    theta = reparam.to_theta(x)
    if profile:
        t = point(x)
        s2 = math.exp(_profile_parts(t)[1])
        theta = (s2, t[1], t[2], t[3] * s2)
    return dict(log=log, evals=pre_calls + res.nfev - 1, iters=res.nit - 1, theta=theta, logL=-res.fun,
                converged=int(res.nit - 1 < max_iter))


CASES = [
    # profile, start, step, tol, max_iter, nugget floor, band of failing ell
    (False, None, 1.0, 1e-4, 400, 0.0, 0.0),                   # the paper's start, default tolerance
    (False, None, 1.0, 1e-6, 400, 1e-6, 0.0),                  # start back-off, failed vertices in the search
    (False, (1.0, 0.1, 0.5, 0.01), 0.5, 1e-5, 25, 0.0, 0.0),   # stops at max_iter
    (True, (1.0, 0.1, 0.5, 0.01), 1.0, 1e-6, 400, 0.0, 0.0),   # variance profiled out
    (True, None, 1.0, 1e-6, 400, 1e-5, 0.0),                   # profiled, with back-off
    (False, (1.0, 0.1, 0.5, 1e-5), 3.0, 1e-4, 400, 5e-4, 0.0),  # large steps against the infeasible region
    (False, None, 1.0, 1e-4, 400, 0.0, 0.18),                  # contractions into the band: shrinks
    (True, None, 1.0, 1e-4, 400, 0.0, 0.35),
]


@pytest.mark.parametrize("profile,start,step,tol,max_iter,floor,band", CASES)
def test_nelder_mead_matches_scipy(driver, profile, start, step, tol, max_iter, floor, band):
    evals, got = _run(driver, profile, start, step, tol, max_iter, floor, band)
    ref = _scipy_search(profile, start, step, tol, max_iter, floor, band)
    assert got is not None
    print(f"profile={profile} start={start}: {got['evals']} evaluations, {got['iters']} iterations, "
          f"{got['failed']} failed, status {got['status']}")
    assert len(evals) == len(ref["log"])
    for a, b in zip(evals, ref["log"]):
        xa, xb = reparam.from_theta(a), reparam.from_theta(b)
        assert max(abs(p - q) for p, q in zip(xa, xb)) <= 1e-9, (a, b)
    assert got["evals"] == ref["evals"] and got["iters"] == ref["iters"]
    assert got["failed"] == got["evals"] - len(evals)
    assert got["converged"] == ref["converged"]
    assert got["status"] == (0 if ref["converged"] else 6)
    assert all(abs(a - b) <= 1e-8 * abs(b) for a, b in zip(got["theta"], ref["theta"]))
    assert abs(got["logL"] - ref["logL"]) <= 1e-9 * max(1.0, abs(ref["logL"]))
    if floor > 0:
        assert got["failed"] > 0


def _run_lines(exe, profile, start, step, tol, max_iter, floor, band, stop_at=0):
    s = start if start is not None else (0, 0, 0, 0)
    args = [exe, str(int(profile))] + [repr(float(v)) for v in s] + [repr(step), repr(tol), str(max_iter), repr(floor),
                                                                     repr(band)]
    if stop_at:
        args.append(str(stop_at))
    r = subprocess.run(args, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout.splitlines()


@pytest.mark.parametrize("case", [CASES[0], CASES[1], CASES[3], CASES[4], CASES[6], CASES[7]])
@pytest.mark.parametrize("stop_at", [1, 10, 37])
def test_resume_equals_uninterrupted(driver, case, stop_at):
    """hmle_fit_resumable stopped after stop_at iterations and continued from
    its checkpoint evaluates the same points as the uninterrupted fit and
    returns the same estimate and counts, bit for bit; a call with the final
    checkpoint evaluates nothing and returns the same; the checkpoint is
    refused by the other kind of search."""
    full = _run_lines(driver, *case)
    res = _run_lines(driver, *case, stop_at=stop_at)
    assert [l for l in res if l.startswith("eval")] == [l for l in full if l.startswith("eval")]
    want = next(l for l in full if l.startswith("result")).split()[1:]
    stopped = next(l for l in res if l.startswith("stopped")).split()
    iters_full = int(want[6])
    if stop_at < iters_full:
        assert int(stopped[1]) == 6 and int(stopped[3]) == stop_at     # E_NOCONV at the stop
    assert next(l for l in res if l.startswith("result")).split()[1:] == want
    assert next(l for l in res if l.startswith("again")).split()[1:] == want
    assert next(l for l in res if l.startswith("mismatch")).split()[1] == "1"   # HMLE_E_INVALID
    assert next(l for l in res if l.startswith("otherdata")).split()[1] == "1"  # another z: refused



@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("count", [2, 3, 4])
def test_batched_fit_equals_sequential(driver, case, count):
    """hmle_fit_batch (the same iteration, the points an iteration may need
    evaluated `count` at a time, speculatively) returns exactly the estimate,
    log-likelihood and counts of hmle_fit, in fewer batched rounds than
    evaluations."""
    s = case[1] if case[1] is not None else (0, 0, 0, 0)
    args = [driver, str(int(case[0]))] + [repr(float(v)) for v in s] + [repr(case[2]), repr(case[3]), str(case[4]),
                                                                        repr(case[5]), repr(case[6]), "0", str(count)]
    r = subprocess.run(args, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.splitlines()
    seq = next(l for l in lines if l.startswith("result")).split()[1:]
    bat = next(l for l in lines if l.startswith("batch")).split()[1:]
    assert bat[:10] == seq
    evals, rounds = int(bat[5]), int(bat[10])
    assert 0 < rounds < evals
