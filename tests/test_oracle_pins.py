"""Pins of the oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms of the Matern function (eq. 2), a different special-function library
(mpmath), the small-argument limit, explicit n=1 and n=2 likelihoods, an LU
log-determinant, an independent state-space likelihood for collinear points,
limits and invariances of eq. (1). ``test_mutations_are_caught`` plants
plausible mistakes in the oracle and checks that the pins catch each one.
"""
import math

import mpmath
import numpy as np
import pytest

import synth
from oracle import dense, kalman, matern, reparam

RNG_SUB = 100


def _rng(k=0):
    return synth.rng_for(synth.W_TESTS, RNG_SUB + k)


XS = np.concatenate([np.geomspace(1e-8, 1e-2, 7), np.linspace(0.02, 5.0, 40), np.geomspace(5.0, 600.0, 9)])


# ---------------------------------------------------------------- Matern ----
def check_closed_forms(m=matern.matern):
    sigma2, ell = 1.7, 0.3
    h = XS * ell
    x = h / ell
    got = {nu: m(h, sigma2, ell, nu) for nu in (0.5, 1.5, 2.5)}
    want = {0.5: sigma2 * np.exp(-x),
            1.5: sigma2 * (1.0 + x) * np.exp(-x),
            2.5: sigma2 * (1.0 + x + x * x / 3.0) * np.exp(-x)}
    small = x <= 5.0
    for nu in want:
        # exp(-x) at large x carries a relative error of about x * 2^-53.
        np.testing.assert_allclose(got[nu][small], want[nu][small], rtol=2e-14, atol=0)
        np.testing.assert_allclose(got[nu], want[nu], rtol=1e-13, atol=1e-300)


def check_mpmath(m=matern.matern):
    mpmath.mp.dps = 30
    sigma2, ell = 0.9, 0.07
    for nu in (0.05, 0.3, 0.5, 0.83, 1.0, 1.37, 2.0, 3.3, 5.0, 8.0):
        for x in (1e-6, 1e-3, 0.1, 0.5, 1.0, 2.0, 3.7, 10.0, 50.0, 300.0):
            xm = mpmath.mpf(x)
            ref = (mpmath.mpf(sigma2) * mpmath.power(2, 1 - mpmath.mpf(nu)) / mpmath.gamma(nu)
                   * mpmath.power(xm, nu) * mpmath.besselk(nu, xm))
            got = float(m(np.array([x * ell]), sigma2, ell, nu)[0])
            assert abs(got - float(ref)) <= 1e-13 * abs(float(ref)) + 1e-300, (nu, x, got, float(ref))


def check_small_x_limit(m=matern.matern):
    # x^nu K_nu(x) -> 2^(nu-1) Gamma(nu) as x -> 0 (DLMF 10.30.2), so M -> sigma^2.
    for nu in (0.6, 1.0, 2.5, 6.0):
        v = float(m(np.array([1e-9]), 2.3, 1.0, nu)[0])
        assert abs(v / 2.3 - 1.0) < 1e-6, (nu, v)
    assert float(m(np.array([0.0]), 2.3, 0.5, 0.77)[0]) == 2.3


def check_recurrence(m=matern.matern):
    # DLMF 10.29.1: K_{nu+1}(x) = K_{nu-1}(x) + (2 nu / x) K_nu(x); in terms of
    # g_nu(x) = M_nu(x) Gamma(nu) / (sigma^2 2^(1-nu) x^nu) = K_nu(x).
    def K(nu, x):
        return float(m(np.array([x]), 1.0, 1.0, nu)[0]) * math.gamma(nu) / (2.0 ** (1 - nu) * x ** nu)
    for nu in (1.2, 2.0, 3.7):
        for x in (0.3, 1.0, 4.0):
            lhs = K(nu + 1, x)
            rhs = K(nu - 1, x) + 2 * nu / x * K(nu, x)
            assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_matern_closed_forms():
    check_closed_forms()


def test_matern_mpmath():
    check_mpmath()


def test_matern_small_x_limit():
    check_small_x_limit()


def test_matern_recurrence():
    check_recurrence()


def test_matern_monotone_positive():
    h = np.linspace(0.0, 3.0, 400)
    for nu in (0.1, 0.5, 1.0, 2.2, 7.0):
        v = matern.matern(h, 1.3, 0.2, nu)
        assert np.all(v > 0) or np.all(v[-5:] >= 0)
        assert np.all(np.diff(v) <= 0)
        assert v[0] == 1.3


# ------------------------------------------------------- log-likelihood ----
def check_n1(loglik=dense.loglik):
    theta = (1.4, 0.2, 0.8, 0.05)
    z = np.array([0.7])
    got = loglik(np.array([[0.3, 0.4]]), z, theta)[0]
    s = theta[0] + theta[3]
    want = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(s) - z[0] ** 2 / (2 * s)
    assert abs(got - want) <= 1e-14 * abs(want)


def check_n2(loglik=dense.loglik):
    sigma2, ell, tau2 = 1.1, 0.25, 0.03
    pts = np.array([[0.1, 0.2], [0.4, 0.6]])
    h = 0.5
    z = np.array([0.3, -1.2])
    a = sigma2 + tau2
    b = sigma2 * math.exp(-h / ell)               # nu = 1/2 closed form
    det = a * a - b * b
    quad = (a * z[0] ** 2 - 2 * b * z[0] * z[1] + a * z[1] ** 2) / det
    want = -math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * quad
    got, gdet, gquad = loglik(pts, z, (sigma2, ell, 0.5, tau2))
    assert abs(got - want) <= 1e-13 * abs(want)
    assert abs(gdet - math.log(det)) <= 1e-13 * abs(math.log(det)) + 1e-15
    assert abs(gquad - quad) <= 1e-13 * abs(quad)


def check_slogdet(loglik=dense.loglik):
    rng = _rng(1)
    pts = synth.uniform_points(300, 2, rng)
    theta = (1.0, 0.1, 1.3, 0.01)
    C = dense.covariance(pts, theta)
    sign, ld = np.linalg.slogdet(C)       # LU route
    z = synth.standard_normal(300, rng)
    got = loglik(pts, z, theta)
    assert sign > 0
    assert abs(got[1] - ld) <= 1e-10 * abs(ld)
    quad = float(z @ np.linalg.solve(C, z))
    assert abs(got[2] - quad) <= 1e-9 * abs(quad)


def check_kalman(loglik=dense.loglik):
    rng = _rng(2)
    pts, t, _u = synth.collinear_points(400, 2, rng)
    z = synth.standard_normal(400, rng)
    for nu in (0.5, 1.5):
        theta = (1.2, 0.15, nu, 1e-3)
        k = kalman.loglik_collinear(t, z, theta)
        d = loglik(pts, z, theta)[0]
        assert abs(k - d) <= 1e-11 * abs(k), (nu, k, d)


def check_tiny_range_limit(loglik=dense.loglik):
    # ell far below the minimum spacing: every off-diagonal entry underflows
    # to 0 and C = (sigma^2 + tau^2) I.
    rng = _rng(3)
    pts = synth.jittered_grid_points(20, 20, rng)
    z = synth.standard_normal(400, rng)
    sigma2, tau2 = 0.8, 0.1
    ell = (0.2 / 20) / 800.0
    got = loglik(pts, z, (sigma2, ell, 0.5, tau2))[0]
    s = sigma2 + tau2
    want = -200 * math.log(2 * math.pi * s) - float(z @ z) / (2 * s)
    assert abs(got - want) <= 1e-13 * abs(want)


def check_quad_identity(loglik=dense.loglik):
    # Z = C w  =>  Z^T C^{-1} Z = w^T Z.
    rng = _rng(4)
    pts = synth.uniform_points(250, 3, rng)
    theta = (0.7, 0.3, 0.9, 0.02)
    w = synth.standard_normal(250, rng)
    C = dense.covariance(pts, theta)
    z = C @ w
    got = loglik(pts, z, theta)[2]
    assert abs(got - float(w @ z)) <= 1e-9 * abs(float(w @ z))


def test_loglik_n1():
    check_n1()


def test_loglik_n2():
    check_n2()


def test_loglik_slogdet():
    check_slogdet()


def test_loglik_kalman():
    check_kalman()


def test_loglik_tiny_range_limit():
    check_tiny_range_limit()


def test_loglik_quad_identity():
    check_quad_identity()


def test_loglik_scale_invariance():
    rng = _rng(5)
    pts = synth.uniform_points(300, 2, rng)
    z = synth.standard_normal(300, rng)
    theta = (1.0, 0.12, 1.1, 0.01)
    a = 3.7
    l1 = dense.loglik(pts, z, theta)[0]
    l2 = dense.loglik(pts, math.sqrt(a) * z, (a * theta[0], theta[1], theta[2], a * theta[3]))[0]
    assert abs(l2 - (l1 - 150 * math.log(a))) <= 1e-10 * abs(l1)


def test_loglik_permutation_invariance():
    rng = _rng(6)
    pts = synth.uniform_points(200, 2, rng)
    z = synth.standard_normal(200, rng)
    p = rng.permutation(200)
    theta = (1.0, 0.1, 0.7, 0.01)
    a = dense.loglik(pts, z, theta)[0]
    b = dense.loglik(pts[p], z[p], theta)[0]
    assert abs(a - b) <= 1e-11 * abs(a)


def test_not_spd_detected():
    pts = np.array([[0.5, 0.5], [0.5, 0.5], [0.1, 0.9]])   # duplicated point, no nugget
    with pytest.raises(dense.NotSPD):
        dense.cholesky(dense.covariance(pts, (1.0, 0.3, 0.5, 0.0)) - 1e-3 * np.eye(3))


# ----------------------------------------------------------- reparam -------
def test_reparam_paper_start():
    # Section 5.1: sigma = 2/1.1^2, ell = 1/1.5^2, nu = 1/1.2, tau = 2^-15.
    th = reparam.to_theta(reparam.PAPER_START)
    assert abs(th[0] - (2 / 1.21) ** 2) < 1e-15
    assert abs(th[1] - 1 / 2.25) < 1e-15
    assert abs(th[2] - 1 / 1.2) < 1e-15
    assert th[3] == 2.0 ** -30
    back = reparam.from_theta(th)
    np.testing.assert_allclose(back, reparam.PAPER_START, rtol=1e-12)


# ------------------------------------------------------- mutations ----------
ALL_CHECKS = [check_closed_forms, check_mpmath, check_small_x_limit, check_recurrence]
LL_CHECKS = [check_n1, check_n2, check_slogdet, check_kalman, check_tiny_range_limit, check_quad_identity]


def _mut_matern(kind):
    base = matern.matern

    def m(h, sigma2, ell, nu):
        if kind == "no_2pow":
            return base(h, sigma2, ell, nu) / 2.0 ** (1.0 - nu)
        if kind == "nu_plus":
            return base(h, sigma2, ell, nu + 1e-3)
        if kind == "sqrt2nu":
            return base(np.asarray(h) * math.sqrt(2 * nu), sigma2, ell, nu)
        if kind == "sigma_not_squared":
            return base(h, math.sqrt(sigma2), ell, nu)
        raise AssertionError
    return m


def _mut_loglik(kind):
    def ll(pts, z, theta):
        C = dense.covariance(pts, theta)
        if kind == "no_nugget":
            C[np.diag_indices(len(z))] -= theta[3]
        if kind == "nugget_everywhere":
            C += theta[3]
        if kind == "transpose_solve":
            L = dense.cholesky(C)
            n = len(z)
            logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
            v = np.linalg.solve(L.T, z)
            quad = float(v @ v)
            return -0.5 * n * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad, logdet, quad
        L = dense.cholesky(C)
        logL, logdet, quad = dense.loglik_from_factor(L, z)
        if kind == "logdet_once":
            logdet = logdet / 2.0
            logL = -0.5 * len(z) * math.log(2 * math.pi) - 0.5 * logdet - 0.5 * quad
        if kind == "quad_sign":
            logL = logL + quad
        return logL, logdet, quad
    return ll


@pytest.mark.parametrize("kind", ["no_2pow", "nu_plus", "sqrt2nu", "sigma_not_squared"])
def test_mutations_are_caught_matern(kind):
    m = _mut_matern(kind)
    failed = 0
    for chk in ALL_CHECKS:
        try:
            chk(m)
        except AssertionError:
            failed += 1
    assert failed >= 1, f"mutation {kind} not caught"


@pytest.mark.parametrize("kind", ["no_nugget", "nugget_everywhere", "transpose_solve", "logdet_once", "quad_sign"])
def test_mutations_are_caught_loglik(kind):
    ll = _mut_loglik(kind)
    failed = 0
    for chk in LL_CHECKS:
        try:
            chk(ll)
        except (AssertionError, dense.NotSPD, np.linalg.LinAlgError):
            failed += 1
    assert failed >= 1, f"mutation {kind} not caught"
