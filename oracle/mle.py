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


def fit(pts, z, x0=reparam.PAPER_START, max_iter: int = 400, tol: float = 1e-4):
    x0 = np.asarray(x0, dtype=np.float64)
    simplex = np.vstack([x0] + [x0 + np.eye(4)[i] for i in range(4)])
    res = optimize.minimize(negloglik, x0, args=(pts, z), method="Nelder-Mead",
                            options={"initial_simplex": simplex, "xatol": tol, "fatol": tol,
                                     "maxiter": max_iter, "maxfev": 10 * max_iter})
    return {"x": res.x, "theta": reparam.to_theta(res.x), "logL": -float(res.fun),
            "nfev": int(res.nfev), "nit": int(res.nit), "success": bool(res.success)}
