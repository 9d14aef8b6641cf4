"""Kriging prediction, Section 2, eq. (4): the conditional mean of the field
at new locations given the training data,

    Z2 = C21 C11^{-1} Z1,

with C11 the covariance of the training points (eq. (2) plus the nugget on
its diagonal) and C21 the Matern cross-covariance of the new points to the
training points (no nugget: distinct locations); and the prediction-error
measures of Section 3, eqs. (5)-(7): MLOE, MMOM and RMSE. TEST
INFRASTRUCTURE ONLY: plain dense float64 (NumPy / SciPy), the solve by one
Cholesky factor and two triangular substitutions.
"""
from __future__ import annotations

import numpy as np
from scipy import linalg

from . import dense


def predict(pts1, z1, pts2, theta) -> np.ndarray:
    L = dense.cholesky(dense.covariance(pts1, theta))
    v = linalg.solve_triangular(L, np.asarray(z1, dtype=np.float64), lower=True, check_finite=False)
    w = linalg.solve_triangular(L.T, v, lower=False, check_finite=False)
    return dense.cross_covariance(pts2, pts1, theta) @ w


def variance(pts1, pts2, theta) -> np.ndarray:
    """Kriging variance of the field (no nugget) at each new point:
    sigma^2 - c_k^T C11^{-1} c_k with c_k the covariance of new point k with
    the training points, as |L^{-1} c_k|^2 by one triangular substitution."""
    L = dense.cholesky(dense.covariance(pts1, theta))
    C12 = dense.cross_covariance(pts1, pts2, theta)
    V = linalg.solve_triangular(L, C12, lower=True, check_finite=False)
    return theta[0] - np.sum(V * V, axis=0)


def expected_sq_error(pts1, pts2, theta_pred, theta_true, noisy: bool = True) -> np.ndarray:
    """Mean squared error, under the model theta_true, of the kriging
    prediction made with theta_pred, at each new point (the expectations in
    eqs. (5) and (6)). The predictor is w^T Z1 with the weights of eq. (4)
    for theta_pred, w = C11(pred)^{-1} c(pred); the target Z is the value at
    the new point, an observation with its nugget when ``noisy`` (a held-out
    datum), else the field. With Z Gaussian of mean zero under theta_true,
        E (w^T Z1 - Z)^2 = w^T C11(true) w - 2 w^T c(true) + Var_true(Z).
    """
    pts1 = np.asarray(pts1, dtype=np.float64)
    pts2 = np.asarray(pts2, dtype=np.float64)
    Lp = dense.cholesky(dense.covariance(pts1, theta_pred))
    Cp = dense.cross_covariance(pts1, pts2, theta_pred)
    W = linalg.cho_solve((Lp, True), Cp, check_finite=False)          # n x M prediction weights
    Ct = dense.covariance(pts1, theta_true)
    ct = dense.cross_covariance(pts1, pts2, theta_true)
    var_z = theta_true[0] + (theta_true[3] if noisy else 0.0)
    return np.sum(W * (Ct @ W), axis=0) - 2.0 * np.sum(W * ct, axis=0) + var_z


def mloe_mmom(pts1, pts2, theta_est, theta_true, noisy: bool = True) -> tuple[float, float]:
    """Eqs. (5) and (6) over the new points: with a = the estimated model and
    t = the true one,
        MLOE = mean( E_t(Za - Z)^2 / E_t(Zt - Z)^2 - 1 ),
        MMOM = mean( E_a(Za - Z)^2 / E_t(Za - Z)^2 - 1 ),
    Za, Zt the kriging predictions with the estimated and the true
    parameters, E_t, E_a expectations under the true and the estimated model."""
    e_ta = expected_sq_error(pts1, pts2, theta_est, theta_true, noisy)
    e_tt = expected_sq_error(pts1, pts2, theta_true, theta_true, noisy)
    e_aa = expected_sq_error(pts1, pts2, theta_est, theta_est, noisy)
    return float(np.mean(e_ta / e_tt - 1.0)), float(np.mean(e_aa / e_ta - 1.0))


def rmse(pred, z) -> float:
    """Eq. (7): root mean square of the prediction errors at the test points."""
    d = np.asarray(pred, dtype=np.float64) - np.asarray(z, dtype=np.float64)
    return float(np.sqrt(np.mean(d * d)))
