"""Pins of the profiled-variance log-likelihood of the oracle (the maximum of
eq. (1) over sigma^2 with tau^2 = r sigma^2): it equals the plain dense
log-likelihood at the closed-form variance, no other variance does better,
rescaling the data by c scales the variance by c^2 and shifts the profile by
-n log c, and the profiled fit reaches the four-parameter optimum."""
import numpy as np
import pytest

import synth
from oracle import dense, mle, reparam


def _field(n, theta, sub):
    rng = synth.rng_for(synth.W_TESTS, sub)
    pts = synth.uniform_points(n, 2, rng)
    w = synth.standard_normal(n, rng)
    return pts, dense.sample(pts, theta, w)


@pytest.mark.parametrize("ell,nu,r", [(0.1, 0.5, 0.02), (0.2, 1.5, 1e-3), (0.05, 1.0, 0.5)])
def test_profile_is_the_maximum_over_the_variance(ell, nu, r):
    pts, z = _field(150, (1.3, 0.12, 0.8, 0.05), 900)
    lp, s2 = mle.profile_loglik(pts, z, ell, nu, r)
    full = lambda v: dense.loglik(pts, z, (v, ell, nu, r * v))[0]
    assert abs(full(s2) - lp) <= 1e-10 * abs(lp)
    for f in (0.5, 0.9, 0.99, 0.999, 1.001, 1.01, 1.1, 2.0):
        assert full(s2 * f) < lp
    # stationarity: the central difference in log sigma^2 vanishes to O(h^2)
    h = 1e-4
    d = (full(s2 * np.exp(h)) - full(s2 * np.exp(-h))) / (2 * h)
    assert abs(d) <= 1e-5 * len(z)


def test_profile_scale_equivariance():
    pts, z = _field(120, (0.7, 0.2, 0.5, 0.01), 901)
    c = 3.7
    lp1, s1 = mle.profile_loglik(pts, z, 0.15, 0.7, 0.03)
    lp2, s2 = mle.profile_loglik(pts, c * z, 0.15, 0.7, 0.03)
    assert s2 == pytest.approx(c * c * s1, rel=1e-12)
    assert lp2 == pytest.approx(lp1 - len(z) * np.log(c), rel=1e-12)


def test_profiled_fit_reaches_the_full_optimum():
    pts, z = _field(200, (1.0, 0.1, 0.8, 0.02), 902)
    start = (float(np.var(z)), 0.12, 1.0, 0.05 * float(np.var(z)))
    x0 = reparam.from_theta(start)
    full = mle.fit(pts, z, x0=x0)
    prof = mle.fit_profile(pts, z, x0=x0)
    l_prof = dense.loglik(pts, z, prof["theta"])[0]
    assert abs(l_prof - prof["logL"]) <= 1e-9 * abs(l_prof)
    assert l_prof >= full["logL"] - 2e-3
    assert prof["nfev"] < full["nfev"]
