"""Maximum-likelihood reference (Section 2, "Maximization of the
log-likelihood"; Section 5.1 for the coordinates and the start point).

The paper names a Brent-Dekker routine, which is one-dimensional; for the
four parameters this reference uses SciPy's Nelder-Mead on -L in the
transformed coordinates of Section 5.1, with the initial simplex x0, x0+e_i,
tolerance 1e-4 on the simplex and on f, and at most 400 iterations
(Section 2). A point outside the parameter box, or whose covariance matrix
has no Cholesky factor, gets f = +inf.
"""
from __future__ import annotations

import numpy as np
from scipy import optimize

from . import dense, reparam

BOX = {"sigma2": (1e-6, 1e6), "ell": (1e-4, 10.0), "nu": (0.05, 8.0), "tau2": (0.0, 1e3)}


def in_box(theta) -> bool:
    s2, ell, nu, t2 = theta
    return (BOX["sigma2"][0] <= s2 <= BOX["sigma2"][1] and BOX["ell"][0] <= ell <= BOX["ell"][1]
            and BOX["nu"][0] <= nu <= BOX["nu"][1] and BOX["tau2"][0] <= t2 <= BOX["tau2"][1])


def negloglik(x, pts, z) -> float:
    theta = reparam.to_theta(x)
    if not in_box(theta):
        return np.inf
    try:
        return -dense.loglik(pts, z, theta)[0]
    except dense.NotSPD:
        return np.inf


def fit(pts, z, x0=reparam.PAPER_START, max_iter: int = 400, tol: float = 1e-4, objective=None):
    """Nelder-Mead on f = objective(x, pts, z) (default: -L by negloglik) from
    the simplex x0, x0 + e_i in the Section 5.1 coordinates; logL = -f at the
    minimiser found."""
    f = negloglik if objective is None else objective
    x0 = np.asarray(x0, dtype=np.float64)
    simplex = np.vstack([x0] + [x0 + np.eye(4)[i] for i in range(4)])
    res = optimize.minimize(f, x0, args=(pts, z), method="Nelder-Mead",
                            options={"initial_simplex": simplex, "xatol": tol, "fatol": tol,
                                     "maxiter": max_iter, "maxfev": 10 * max_iter})
    return {"x": res.x, "theta": reparam.to_theta(res.x), "logL": -float(res.fun),
            "nfev": int(res.nfev), "nit": int(res.nit), "success": bool(res.success)}


# ---------------------------------------------------- profiled variance -----
# With the nugget written tau^2 = r sigma^2 the covariance is sigma^2 (R + r I),
# R the unit-variance Matern correlation (eq. (2) with sigma^2 = 1). For fixed
# (ell, nu, r), eq. (1) is a function of sigma^2 alone whose maximiser is
# sigma^2 = q / n with q = Z^T (R + r I)^{-1} Z; substituting it gives the
# profile log-likelihood returned here.

def profile_loglik(pts, z, ell: float, nu: float, r: float):
    """(Lp, sigma2_hat) with Lp = -n/2 log(2 pi) - 1/2 log|R + r I| - n/2 log(q/n) - n/2."""
    n = len(z)
    _, logdet, q = dense.loglik(pts, z, (1.0, ell, nu, r))
    s2 = q / n
    return -0.5 * n * np.log(2.0 * np.pi) - 0.5 * logdet - 0.5 * n * np.log(s2) - 0.5 * n, s2


def profile_start(x0):
    """(ell0, nu0, tau0') of a four-parameter start: tau0' codes sqrt(r) = tau / sigma."""
    s2, ell, nu, t2 = reparam.to_theta(x0)
    return np.array([x0[1], x0[2], -np.log(np.sqrt(t2 / s2)) / np.log(2.0)])


def profile_theta(y, s2):
    """Full parameters of a profiled point y = (ell0, nu0, tau0') with variance s2."""
    _, ell, nu, r = reparam.to_theta((0.0, y[0], y[1], y[2]))
    return (s2, ell, nu, r * s2)


def negprofile(y, pts, z) -> float:
    _, ell, nu, r = reparam.to_theta((0.0, y[0], y[1], y[2]))
    if not in_box((1.0, ell, nu, r)):
        return np.inf
    try:
        return -profile_loglik(pts, z, ell, nu, r)[0]
    except dense.NotSPD:
        return np.inf


def fit_profile(pts, z, x0=reparam.PAPER_START, max_iter: int = 400, tol: float = 1e-4, objective=None):
    """SciPy Nelder-Mead on -Lp over (ell0, nu0, tau0'), initial simplex y0, y0 + e_i
    (objective(y, pts, z) replaces negprofile when given)."""
    f = negprofile if objective is None else objective
    y0 = profile_start(np.asarray(x0, dtype=np.float64))
    simplex = np.vstack([y0] + [y0 + np.eye(3)[i] for i in range(3)])
    res = optimize.minimize(f, y0, args=(pts, z), method="Nelder-Mead",
                            options={"initial_simplex": simplex, "xatol": tol, "fatol": tol,
                                     "maxiter": max_iter, "maxfev": 10 * max_iter})
    _, ell, nu, r = reparam.to_theta((0.0, res.x[0], res.x[1], res.x[2]))
    lp, s2 = profile_loglik(pts, z, ell, nu, r)
    return {"y": res.x, "theta": (s2, ell, nu, r * s2), "logL": lp, "nfev": int(res.nfev), "nit": int(res.nit),
            "success": bool(res.success)}
