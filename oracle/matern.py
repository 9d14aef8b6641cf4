"""Matern covariance, Section 1, eq. (2):

    C(h; theta) = sigma^2 / (2^(nu-1) Gamma(nu)) * (h/ell)^nu * K_nu(h/ell)  (+ tau^2 on the diagonal)

Readings (the paper is silent or loose on these):
  * x = h/ell is taken literally, with no sqrt(2 nu) factor; nu=1/2 gives
    sigma^2 exp(-h/ell), nu=3/2 gives sigma^2 (1 + h/ell) exp(-h/ell).
  * At h == 0 the function takes its limit sigma^2 (x^nu K_nu(x) ->
    2^(nu-1) Gamma(nu) as x -> 0).
  * The nugget tau^2 is added on the matrix diagonal only (i == j), never to
    distinct points that happen to coincide; that is done in ``dense``.

Evaluated with SciPy's exponentially scaled K_nu so that large x underflows
smoothly instead of producing inf * 0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def matern(h, sigma2: float, ell: float, nu: float) -> np.ndarray:
    """Matern covariance (no nugget) at distances ``h`` (any shape, float64)."""
    h = np.asarray(h, dtype=np.float64)
    out = np.full(h.shape, float(sigma2))
    pos = h > 0.0
    if np.any(pos):
        x = h[pos] / ell
        # log of sigma^2 * 2^(1-nu)/Gamma(nu) * x^nu * exp(-x); times K_nu(x) e^x
        logpre = (math.log(sigma2) + (1.0 - nu) * math.log(2.0) - math.lgamma(nu)
                  + nu * np.log(x) - x)
        out[pos] = np.exp(logpre) * special.kve(nu, x)
    return out
