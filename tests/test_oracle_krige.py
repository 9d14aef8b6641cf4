"""Pins of the dense kriging predictor of the oracle (eq. (4)):

* without a nugget the predictor interpolates: at a training location it
  returns the datum there;
* for the exponential covariance (nu = 1/2) on a line the process is Markov,
  so between two neighbouring training points the predictor depends on those
  two only, with the closed form
      (sinh(d_r / l) z_left + sinh(d_l / l) z_right) / sinh((d_l + d_r) / l),
  d_l, d_r the distances to the left and right neighbour;
* far from every training point (distance >> range) the prediction is zero;
* the predictor is linear in the data.
"""
import numpy as np
import pytest

import synth
from oracle import dense, krige


def _pts(n, sub, dim=2):
    return synth.uniform_points(n, dim, synth.rng_for(synth.W_TESTS, sub))


def test_interpolates_without_nugget():
    pts = _pts(60, 930)
    z = synth.standard_normal(60, synth.rng_for(synth.W_TESTS, 931))
    theta = (1.3, 0.2, 0.5, 0.0)
    pred = krige.predict(pts, z, pts[[3, 17, 42]], theta)
    np.testing.assert_allclose(pred, z[[3, 17, 42]], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("ell", [0.05, 0.3])
def test_markov_exponential_on_a_line(ell):
    rng = synth.rng_for(synth.W_TESTS, 932)
    t = np.sort(rng.random(40))
    pts = np.stack([t, np.zeros_like(t)], axis=1)
    z = rng.standard_normal(40)
    theta = (2.0, ell, 0.5, 0.0)
    for i in (5, 20, 33):
        s = 0.3 * t[i] + 0.7 * t[i + 1]
        dl, dr = s - t[i], t[i + 1] - s
        want = (np.sinh(dr / ell) * z[i] + np.sinh(dl / ell) * z[i + 1]) / np.sinh((dl + dr) / ell)
        got = krige.predict(pts, z, np.array([[s, 0.0]]), theta)[0]
        assert got == pytest.approx(want, rel=1e-8, abs=1e-10)


def test_far_away_is_zero_and_linear():
    pts = _pts(80, 933)
    rng = synth.rng_for(synth.W_TESTS, 934)
    z1, z2 = rng.standard_normal(80), rng.standard_normal(80)
    theta = (1.0, 0.05, 1.0, 0.01)
    far = np.array([[40.0, 40.0]])
    assert abs(krige.predict(pts, z1, far, theta)[0]) < 1e-12
    new = _pts(7, 935)
    a = krige.predict(pts, 2.0 * z1 - 3.0 * z2, new, theta)
    b = 2.0 * krige.predict(pts, z1, new, theta) - 3.0 * krige.predict(pts, z2, new, theta)
    np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("ell", [0.05, 0.3])
def test_variance_markov_bridge_on_a_line(ell):
    """Exponential covariance on a line: given all the data, the variance at a
    point between two neighbours is that of the two-point conditioning,
    sigma^2 (1 - (a^2 + b^2 - 2 a b rho) / (1 - rho^2)), a = e^{-d_l/l},
    b = e^{-d_r/l}, rho = e^{-(d_l + d_r)/l}."""
    rng = synth.rng_for(synth.W_TESTS, 936)
    t = np.sort(rng.random(40))
    pts = np.stack([t, np.zeros_like(t)], axis=1)
    s2 = 1.7
    theta = (s2, ell, 0.5, 0.0)
    for i in (4, 19, 30):
        s = 0.6 * t[i] + 0.4 * t[i + 1]
        dl, dr = s - t[i], t[i + 1] - s
        a, b, rho = np.exp(-dl / ell), np.exp(-dr / ell), np.exp(-(dl + dr) / ell)
        want = s2 * (1.0 - (a * a + b * b - 2 * a * b * rho) / (1.0 - rho * rho))
        got = krige.variance(pts, np.array([[s, 0.0]]), theta)[0]
        assert got == pytest.approx(want, rel=1e-8, abs=1e-12)


def test_variance_limits_and_monotone():
    pts = _pts(90, 937)
    theta = (1.4, 0.1, 1.0, 0.0)
    v_train = krige.variance(pts, pts[[2, 50]], theta)
    assert np.all(np.abs(v_train) < 1e-8)
    assert krige.variance(pts, np.array([[30.0, 30.0]]), theta)[0] == pytest.approx(1.4, rel=1e-12)
    new = _pts(9, 938)
    th = (1.4, 0.1, 1.0, 0.02)
    full = krige.variance(pts, new, th)
    part = krige.variance(pts[:45], new, th)
    assert np.all(full <= part + 1e-12) and np.all(full > 0)
