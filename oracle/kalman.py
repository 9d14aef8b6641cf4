"""Exact O(n) Gaussian log-likelihood, eq. (1), for locations on a straight
line, where the Matern field with nu = 1/2 or nu = 3/2 is a linear
state-space (Markov) process along the line. With x = h/ell as in eq. (2):

  nu = 1/2: M(h) = sigma^2 exp(-lambda h), lambda = 1/ell; one state
            f(t + D) = exp(-lambda D) f(t) + w, var w = sigma^2 (1 - exp(-2 lambda D)).
  nu = 3/2: M(h) = sigma^2 (1 + lambda h) exp(-lambda h); state (f, f'),
            stationary covariance P = diag(sigma^2, lambda^2 sigma^2),
            transition Phi(D) = exp(-lambda D) [[1 + lambda D, D], [-lambda^2 D, 1 - lambda D]],
            process noise Q = P - Phi P Phi^T.

Observations z_k = f(t_k) + e_k with e_k ~ N(0, tau^2). The Kalman filter's
prediction-error decomposition gives L = sum_k -1/2 (log(2 pi S_k) + v_k^2/S_k)
exactly (up to rounding), independently of any covariance matrix. It pins the
dense oracle at small n and stands in for it at large n.
"""
from __future__ import annotations

import math

import numpy as np


def loglik_collinear(t, z, theta) -> float:
    """t: positions along the line (any order; sorted internally), z: data in
    the same order as t, theta = (sigma2, ell, nu, tau2) with nu in {0.5, 1.5}."""
    sigma2, ell, nu, tau2 = (float(v) for v in theta)
    t = np.asarray(t, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    order = np.argsort(t, kind="stable")
    t = t[order]
    z = z[order]
    lam = 1.0 / ell
    n = t.shape[0]
    ll = 0.0
    if nu == 0.5:
        m, P = 0.0, sigma2
        for k in range(n):
            if k:
                phi = math.exp(-lam * (t[k] - t[k - 1]))
                m = phi * m
                P = phi * phi * P + sigma2 * (1.0 - phi * phi)
            S = P + tau2
            v = z[k] - m
            ll += -0.5 * (math.log(2.0 * math.pi * S) + v * v / S)
            K = P / S
            m = m + K * v
            P = (1.0 - K) * P
        return ll
    if nu == 1.5:
        Pinf = np.diag([sigma2, lam * lam * sigma2])
        m = np.zeros(2)
        P = Pinf.copy()
        H = np.array([1.0, 0.0])
        for k in range(n):
            if k:
                D = t[k] - t[k - 1]
                e = math.exp(-lam * D)
                Phi = e * np.array([[1.0 + lam * D, D], [-lam * lam * D, 1.0 - lam * D]])
                Q = Pinf - Phi @ Pinf @ Phi.T
                m = Phi @ m
                P = Phi @ P @ Phi.T + Q
            S = float(H @ P @ H) + tau2
            v = z[k] - float(H @ m)
            ll += -0.5 * (math.log(2.0 * math.pi * S) + v * v / S)
            K = (P @ H) / S
            m = m + K * v
            P = P - np.outer(K, H @ P)
            P = 0.5 * (P + P.T)
        return ll
    raise ValueError("collinear exact likelihood exists for nu = 0.5 and 1.5 only")
