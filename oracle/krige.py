"""Kriging prediction, Section 2, eq. (4): the conditional mean of the field
at new locations given the training data,

    Z2 = C21 C11^{-1} Z1,

with C11 the covariance of the training points (eq. (2) plus the nugget on
its diagonal) and C21 the Matern cross-covariance of the new points to the
training points (no nugget: distinct locations). TEST INFRASTRUCTURE ONLY:
plain dense float64 (NumPy / SciPy), the solve by one Cholesky factor and two
triangular substitutions.
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
