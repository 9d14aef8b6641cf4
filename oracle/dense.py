"""Dense float64 reference of the Gaussian log-likelihood, Section 1, eq. (1):

    L(theta) = -n/2 log(2 pi) - 1/2 log|C(theta)| - 1/2 Z^T C(theta)^{-1} Z

computed the plain way: assemble C entry by entry from eq. (2), take its
Cholesky factor C = L L^T, use log|C| = 2 sum_i log L_ii (Section 2, "Storage
and complexity") and Z^T C^{-1} Z = ||L^{-1} Z||^2 via one forward
substitution.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import linalg

from .matern import matern


class NotSPD(Exception):
    """The assembled covariance matrix has no Cholesky factor."""


def pair_distances(pa: np.ndarray, pb: np.ndarray) -> np.ndarray:
    """Euclidean distances |pa_i - pb_j| by direct coordinate differences."""
    pa = np.asarray(pa, dtype=np.float64)
    pb = np.asarray(pb, dtype=np.float64)
    diff = pa[:, None, :] - pb[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=2))


def cross_covariance(pa, pb, theta) -> np.ndarray:
    """Matern covariance block between point sets pa (m,d) and pb (k,d); no nugget."""
    sigma2, ell, nu, _tau2 = theta
    return matern(pair_distances(pa, pb), sigma2, ell, nu)


def covariance(pts, theta, chunk: int = 2048) -> np.ndarray:
    """Full n-by-n covariance C_ij = M(|s_i - s_j|) + tau^2 [i == j]."""
    pts = np.asarray(pts, dtype=np.float64)
    n = pts.shape[0]
    C = np.empty((n, n))
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        C[r0:r1] = cross_covariance(pts[r0:r1], pts, theta)
    C[np.diag_indices(n)] += theta[3]
    return C


def cholesky(C: np.ndarray) -> np.ndarray:
    try:
        return linalg.cholesky(C, lower=True, check_finite=False)
    except linalg.LinAlgError as exc:
        raise NotSPD(str(exc)) from exc


def loglik_from_factor(L: np.ndarray, z) -> tuple[float, float, float]:
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    v = linalg.solve_triangular(L, z, lower=True, check_finite=False)
    quad = math.fsum(v * v) if n <= 64 else float(v @ v)
    logL = -0.5 * n * math.log(2.0 * math.pi) - 0.5 * logdet - 0.5 * quad
    return logL, logdet, quad


def loglik(pts, z, theta) -> tuple[float, float, float]:
    """(logL, logdet, quad) of eq. (1) for locations pts (n,d), data z (n,)."""
    return loglik_from_factor(cholesky(covariance(pts, theta)), z)


def sample(pts, theta, w) -> np.ndarray:
    """Z = L w with C = L L^T: a draw from N(0, C) given standard normals w."""
    L = cholesky(covariance(pts, theta))
    return L @ np.asarray(w, dtype=np.float64)
