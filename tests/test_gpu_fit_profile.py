"""GPU tests of the profiled-variance fit (hmle_fit_opts.profile_variance).

The GPU path searches (ell, nu, r) with sigma^2 in closed form; it is checked
against the oracle's profiled Nelder-Mead (SciPy on the dense profile
likelihood) by the dense log-likelihood at each optimum, its reported logL
against the dense log-likelihood at its own estimate (the profile value equals
eq. (1) at sigma^2 = q / n), and the candidate-batched variant against the
sequential one bit for bit.
"""
import numpy as np
import pytest

import synth
from oracle import dense, mle, reparam

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _field(n, theta, sub):
    rng = synth.rng_for(synth.W_TESTS, sub)
    pts = synth.uniform_points(n, 2, rng)
    w = synth.standard_normal(n, rng)
    return pts, dense.sample(pts, theta, w)


def test_profiled_fit_matches_oracle():
    h = _h()
    pts, z = _field(700, (1.0, 0.1, 0.8, 0.02), 910)
    start = (float(np.var(z)), 0.12, 1.0, 0.05 * float(np.var(z)))
    ref = mle.fit_profile(pts, z, x0=reparam.from_theta(start))
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8) as p:
        fit = p.fit(_cuda(z), start=start, profile_variance=True)
        full = p.fit(_cuda(z), start=start)
    l_gpu = dense.loglik(pts, z, fit.theta)[0]
    print("profiled", fit, "dense logL", l_gpu, "oracle", ref["theta"], ref["logL"], ref["nfev"], "full", full)
    assert fit.converged and fit.status == 0
    assert abs(l_gpu - ref["logL"]) <= 1e-4 * abs(ref["logL"])
    assert abs(fit.logL - l_gpu) <= 1e-6 * abs(l_gpu)
    # the same optimum as the four-parameter search, in fewer evaluations
    assert l_gpu >= dense.loglik(pts, z, full.theta)[0] - 1e-2
    assert fit.evals < full.evals


def test_profiled_batched_equals_sequential():
    h = _h()
    pts, z = _field(800, (1.2, 0.15, 0.6, 0.01), 911)
    start = (float(np.var(z)), 0.1, 1.0, 0.05 * float(np.var(z)))
    dp, dz = _cuda(pts), _cuda(z)
    with h.Problem(dp, leaf_size=64, aca_tol=1e-7) as p:
        seq = p.fit(dz, start=start, profile_variance=True)
    with h.Batch([dp, dp], leaf_size=64, aca_tol=1e-7) as b:
        bat, rounds = b.fit(dz, start=start, profile_variance=True)
    assert bat.theta == seq.theta and bat.logL == seq.logL
    assert (bat.evals, bat.iters, bat.failed_evals, bat.converged) == (seq.evals, seq.iters, seq.failed_evals,
                                                                         seq.converged)
    assert 0 < rounds < bat.evals
