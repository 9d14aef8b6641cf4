"""Parameter transformation of Section 5.1: the optimiser works on
(sigma0, ell0, nu0, tau0) with

    sigma = 2 / 1.1^sigma0,  ell = 1 / 1.5^ell0,  nu = 1 / 1.2^nu0,  tau = 1 / 2^tau0,

so that any real vector maps to positive parameters. sigma and tau are
standard deviations; the covariance uses sigma^2 and tau^2. The paper's
initial guess is (2, 2, 1, 15).
"""
from __future__ import annotations

import math

PAPER_START = (2.0, 2.0, 1.0, 15.0)


def to_theta(x) -> tuple[float, float, float, float]:
    s0, l0, n0, t0 = (float(v) for v in x)
    sigma = 2.0 / 1.1 ** s0
    ell = 1.0 / 1.5 ** l0
    nu = 1.0 / 1.2 ** n0
    tau = 1.0 / 2.0 ** t0
    return (sigma * sigma, ell, nu, tau * tau)


def from_theta(theta) -> tuple[float, float, float, float]:
    sigma2, ell, nu, tau2 = (float(v) for v in theta)
    s0 = math.log(2.0 / math.sqrt(sigma2)) / math.log(1.1)
    l0 = -math.log(ell) / math.log(1.5)
    n0 = -math.log(nu) / math.log(1.2)
    t0 = -math.log(math.sqrt(tau2)) / math.log(2.0)
    return (s0, l0, n0, t0)
