"""GPU tests of the optimiser (hmle_fit), the mixed-precision mode and the
large-n accuracy pins, all through the C ABI."""
import math

import numpy as np
import pytest

import synth
from oracle import dense, kalman, mle, reparam

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _field(n, theta, sub, dim=2):
    rng = synth.rng_for(synth.W_TESTS, sub)
    pts = synth.uniform_points(n, dim, rng)
    w = synth.standard_normal(n, rng)
    return pts, dense.sample(pts, theta, w)


def test_fit_matches_oracle_optimum():
    """Nelder-Mead on the GPU path vs SciPy Nelder-Mead on the dense oracle,
    same start and settings; compared by the oracle's logL at each optimum
    (the likelihood is flat with several near-optima, so theta is not compared)."""
    h = _h()
    theta_true = (1.0, 0.1, 0.8, 0.02)
    pts, z = _field(700, theta_true, 700)
    start = (float(np.var(z)), 0.12, 1.0, 0.05 * float(np.var(z)))
    ref = mle.fit(pts, z, x0=reparam.from_theta(start), max_iter=400, tol=1e-4)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8) as p:
        fit = p.fit(_cuda(z), start=start, max_iter=400, tol=1e-4)
    l_gpu = dense.loglik(pts, z, fit.theta)[0]
    l_ref = ref["logL"]
    print("gpu", fit, "logL(oracle)", l_gpu, "oracle fit", ref["theta"], l_ref, ref["nfev"])
    assert fit.converged and fit.status == 0
    assert abs(l_gpu - l_ref) <= 1e-4 * abs(l_ref)
    assert abs(fit.logL - l_gpu) <= 1e-6 * abs(l_gpu)


def test_fit_paper_start_with_backoff_and_noconv():
    h = _h()
    theta_true = (1.0, 0.1, 0.5, 0.01)
    pts, z = _field(500, theta_true, 701)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8) as p:
        fit = p.fit(_cuda(z), start=None, max_iter=3)
        assert fit.status == h.HMLE_E_NOCONV and not fit.converged and fit.iters == 3
        assert math.isfinite(fit.logL) and fit.evals >= 5


@pytest.mark.parametrize("nu", [0.5, 1.0])
def test_mixed_precision_reported(nu):
    """float32 assembly / low-rank arithmetic / near-field updates with float64
    diagonal leaves, log-det and quadratic form; the deviation is reported and
    gated only loosely (finite, positive definite, 1e-2 relative)."""
    h = _h()
    rng = synth.rng_for(synth.W_SMALL_UNIFORM)
    pts = synth.uniform_points(2000, 2, rng)
    w = synth.standard_normal(2000, rng)
    theta = (1.0, 0.1, nu, 0.01)
    z = dense.sample(pts, theta, w)
    ref = dense.loglik(pts, z, theta)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-6, precision=h.MIXED) as p:
        got = p.eval(theta, _cuda(z))
    rel = abs(got[0] - ref[0]) / abs(ref[0])
    print(f"mixed nu={nu}: logL {got[0]:.6f} vs {ref[0]:.6f}, |dlogL| {abs(got[0]-ref[0]):.3e}, rel {rel:.3e}")
    assert math.isfinite(got[0]) and rel <= 1e-2


@pytest.mark.parametrize("n,nu", [(64000, 0.5), (64000, 1.5), (256000, 0.5)])
def test_collinear_kalman_pin_large_n(n, nu):
    """Points on a segment: the Matern field with nu = 1/2 or 3/2 is Markov
    along the line, so the exact logL is a Kalman filter; far-field blocks are
    exactly rank 1 or 2, and the H path must match to 1e-8 relative."""
    h = _h()
    rng = synth.rng_for(synth.W_TESTS, 800 + n)
    pts, t, _u = synth.collinear_points(n, 2, rng, length=1.0)
    z = synth.standard_normal(n, rng)
    theta = (1.0, 0.05, nu, 1e-3)
    ref = kalman.loglik_collinear(t, z, theta)
    with h.Problem(_cuda(pts), leaf_size=128, aca_tol=1e-10, max_rank=16) as p:
        got = p.eval(theta, _cuda(z))
        st = p.stats()
    rel = abs(got[0] - ref) / abs(ref)
    print(f"collinear n={n} nu={nu}: H {got[0]:.8f} Kalman {ref:.8f} rel {rel:.3e} ranks {st}")
    assert rel <= 1e-8
