"""Pins of the oracle's exact covariance-vector product (oracle/matvec.c):
against the dense covariance matrix of the pinned oracle (2-D and 3-D, both
closed-form smoothness values, duplicated points where h = 0 gives sigma^2),
the symmetry v . (C w) = w . (C v), and the quadratic-form identity it is
used for: with Z = C w, Z^T C^{-1} Z = w^T Z; the nugget's contribution on
its own."""
import numpy as np
import pytest

import synth
from oracle import dense, matvec


@pytest.mark.parametrize("dim,nu", [(2, 0.5), (2, 1.5), (3, 0.5), (3, 1.5)])
def test_matvec_equals_dense_product(dim, nu):
    rng = synth.rng_for(synth.W_TESTS, 961 + dim)
    pts = synth.uniform_points(1500, dim, rng)
    pts[100:110] = pts[0]                      # duplicated points: h = 0
    theta = (1.3, 0.1, nu, 0.02)
    w = rng.standard_normal(1500)
    y = matvec.cov_matvec(pts, theta, w)
    C = dense.covariance(pts, theta)
    ref = C @ w
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    v = rng.standard_normal(1500)
    assert abs(v @ y - w @ matvec.cov_matvec(pts, theta, v)) <= 1e-11 * abs(v @ y)
    # several right-hand sides in one pass give the single products
    W = rng.standard_normal((1500, 3))
    Y = matvec.cov_matvec(pts, theta, W)
    assert np.abs(Y - C @ W).max() <= 1e-13 * np.abs(C @ W).max()
    # the quadratic-form identity the large-n pin relies on
    z = y
    L = dense.cholesky(C)
    quad = dense.loglik_from_factor(L, z)[2]
    assert abs(quad - w @ z) <= 1e-8 * abs(w @ z)


def test_matvec_nugget_is_seen():
    rng = synth.rng_for(synth.W_TESTS, 966)
    pts = synth.uniform_points(300, 2, rng)
    w = rng.standard_normal(300)
    a = matvec.cov_matvec(pts, (1.0, 0.1, 0.5, 0.0), w)
    b = matvec.cov_matvec(pts, (1.0, 0.1, 0.5, 0.3), w)
    assert np.allclose(b - a, 0.3 * w, rtol=0, atol=1e-13)


def test_matvec_refuses_other_smoothness():
    with pytest.raises(ValueError):
        matvec.cov_matvec(np.zeros((3, 2)), (1.0, 0.1, 1.0, 0.0), np.ones(3))
