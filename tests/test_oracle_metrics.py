"""Pins of the oracle's prediction-error measures, Section 3, eqs. (5)-(7)
(oracle/krige.py: expected_sq_error, mloe_mmom, rmse):

* Monte Carlo: joint draws of training data and targets from the true model,
  predicted with the estimated parameters by the (separately pinned) kriging
  predictor; the sample mean of the squared errors must match the closed form
  within five standard errors, for held-out observations (with nugget) and for
  the field; planted mistakes in the closed form fail this check;
* the exponential covariance on a line is Markov, so a prediction between two
  neighbours uses those two only and its error under another range has a
  three-variable closed form;
* estimate = truth gives MLOE = MMOM = 0; scaling sigma^2 and tau^2 by c
  leaves the predictor unchanged, so MLOE = 0 and MMOM = c - 1 exactly;
* the true-model predictor is optimal under the true model, so MLOE >= 0;
* at estimate = truth the error of the field is the kriging variance, and that
  of an observation adds the nugget;
* RMSE on a hand-worked example.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, krige

THETA_T = (1.0, 0.1, 0.5, 0.02)
THETA_A = (1.4, 0.16, 0.7, 0.005)


def _pts(n, sub):
    return synth.uniform_points(n, 2, synth.rng_for(synth.W_TESTS, sub))


def _mc_zscores(fn, noisy, n_draws=200_000):
    """Largest |mean - closed form| / standard error over the new points."""
    p1, p2 = _pts(30, 960), _pts(5, 961)
    allp = np.concatenate([p1, p2])
    K = dense.covariance(allp, THETA_T)
    if not noisy:
        K[30:, 30:] -= THETA_T[3] * np.eye(5)     # the targets are field values
    L = np.linalg.cholesky(K)
    rng = synth.rng_for(synth.W_TESTS, 962)
    S = L @ rng.standard_normal((35, n_draws))
    pred = krige.predict(p1, S[:30], p2, THETA_A)
    sq = (pred - S[30:]) ** 2
    mean, se = sq.mean(axis=1), sq.std(axis=1) / math.sqrt(n_draws)
    want = fn(p1, p2, THETA_A, THETA_T, noisy)
    return float(np.max(np.abs(mean - want) / se))


@pytest.mark.parametrize("noisy", [True, False])
def test_expected_error_matches_monte_carlo(noisy):
    z = _mc_zscores(krige.expected_sq_error, noisy)
    print("noisy", noisy, "largest z-score", z)
    assert z <= 5.0


def test_monte_carlo_rejects_planted_mistakes():
    def cross_once(p1, p2, ta, tt, noisy):        # cross term counted once
        W = np.linalg.solve(dense.covariance(p1, ta), dense.cross_covariance(p1, p2, ta))
        return (np.sum(W * (dense.covariance(p1, tt) @ W), axis=0)
                - np.sum(W * dense.cross_covariance(p1, p2, tt), axis=0) + tt[0] + (tt[3] if noisy else 0))

    def no_nugget(p1, p2, ta, tt, noisy):          # observation variance without its nugget
        return krige.expected_sq_error(p1, p2, ta, tt, noisy=False)

    def swapped(p1, p2, ta, tt, noisy):            # the two models exchanged
        return krige.expected_sq_error(p1, p2, tt, ta, noisy)

    assert _mc_zscores(cross_once, True) > 5.0
    assert _mc_zscores(no_nugget, True) > 5.0
    assert _mc_zscores(swapped, True) > 5.0


@pytest.mark.parametrize("ell_t,ell_a", [(0.05, 0.1), (0.3, 0.12)])
def test_markov_line_closed_form(ell_t, ell_a):
    rng = synth.rng_for(synth.W_TESTS, 963)
    t = np.sort(rng.random(40))
    pts = np.stack([t, np.zeros_like(t)], axis=1)
    s2t = 1.3
    tt, ta = (s2t, ell_t, 0.5, 0.0), (0.9, ell_a, 0.5, 0.0)
    for i in (6, 21, 34):
        s = 0.35 * t[i] + 0.65 * t[i + 1]
        dl, dr = s - t[i], t[i + 1] - s
        d = dl + dr
        wl, wr = np.sinh(dr / ell_a) / np.sinh(d / ell_a), np.sinh(dl / ell_a) / np.sinh(d / ell_a)
        rho, a, b = np.exp(-d / ell_t), np.exp(-dl / ell_t), np.exp(-dr / ell_t)
        want = s2t * (1 + wl * wl + wr * wr + 2 * wl * wr * rho - 2 * wl * a - 2 * wr * b)
        got = krige.expected_sq_error(pts, np.array([[s, 0.0]]), ta, tt, noisy=False)[0]
        assert got == pytest.approx(want, rel=1e-7, abs=1e-13)


@pytest.mark.parametrize("noisy", [True, False])
def test_identity_and_scaling(noisy):
    p1, p2 = _pts(70, 964), _pts(9, 965)
    mloe, mmom = krige.mloe_mmom(p1, p2, THETA_T, THETA_T, noisy)
    assert abs(mloe) <= 1e-12 and abs(mmom) <= 1e-12
    for c in (0.5, 3.0):
        scaled = (c * THETA_T[0], THETA_T[1], THETA_T[2], c * THETA_T[3])
        mloe, mmom = krige.mloe_mmom(p1, p2, scaled, THETA_T, noisy)
        assert abs(mloe) <= 1e-10
        assert mmom == pytest.approx(c - 1.0, abs=1e-10)


@pytest.mark.parametrize("noisy", [True, False])
def test_mloe_nonnegative(noisy):
    p1, p2 = _pts(70, 966), _pts(9, 967)
    rng = synth.rng_for(synth.W_TESTS, 968)
    for _ in range(6):
        ta = (float(rng.uniform(0.5, 2)), float(rng.uniform(0.03, 0.3)), float(rng.uniform(0.3, 2)),
              float(rng.uniform(0.001, 0.1)))
        e_ta = krige.expected_sq_error(p1, p2, ta, THETA_T, noisy)
        e_tt = krige.expected_sq_error(p1, p2, THETA_T, THETA_T, noisy)
        assert np.all(e_ta >= e_tt * (1 - 1e-12))
        assert krige.mloe_mmom(p1, p2, ta, THETA_T, noisy)[0] >= -1e-12


def test_error_at_truth_is_the_kriging_variance():
    p1, p2 = _pts(70, 969), _pts(9, 970)
    var = krige.variance(p1, p2, THETA_T)
    np.testing.assert_allclose(krige.expected_sq_error(p1, p2, THETA_T, THETA_T, noisy=False), var,
                               rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(krige.expected_sq_error(p1, p2, THETA_T, THETA_T, noisy=True), var + THETA_T[3],
                               rtol=1e-9, atol=1e-12)


def test_rmse_hand_example():
    assert krige.rmse([1.0, 2.0, 3.0], [1.0, 0.0, 3.0]) == pytest.approx(math.sqrt(4.0 / 3.0), rel=1e-15)
    assert krige.rmse([0.5], [0.5]) == 0.0
