"""GPU parity of the HIP H-MLE path against the float64 dense oracle.

All calls go through the C ABI (libhmle.so) via the thin binding. Tolerances:
  * Matern device function: 1e-13 relative (float64), 2e-6 (float32).
  * n <= leaf size (one dense leaf, no approximation): 1e-12 relative logL.
  * H path, n = 2000, leaf 64, eta 2, eps 1e-6, nu = 1/2: 1e-6 relative logL
    (the accuracy target for small n).
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, matern

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _rel(a, b):
    return abs(a - b) / abs(b)


# ------------------------------------------------------------ Matern -------
@pytest.mark.parametrize("nu", [0.05, 0.3, 0.5, 0.83, 1.0, 1.5, 2.0, 2.5, 3.7, 8.0])
def test_matern_fp64(nu):
    h = _h()
    x = np.concatenate([[0.0], np.geomspace(1e-7, 1, 40), np.linspace(1.0, 40, 60), np.geomspace(40, 690, 20)])
    ell, sigma2 = 0.13, 1.7
    dist = x * ell
    got = h.matern(_cuda(dist), (sigma2, ell, nu, 0.0)).cpu().numpy()
    want = matern.matern(dist, sigma2, ell, nu)
    big = want > 1e-290
    err = np.abs(got[big] - want[big]) / want[big]
    assert err.max() <= 1e-13, (nu, float(err.max()), x[big][np.argmax(err)])
    assert got[0] == sigma2


@pytest.mark.parametrize("nu", [0.3, 0.5, 1.0, 1.5, 2.7])
def test_matern_fp32(nu):
    h = _h()
    x = np.concatenate([[0.0], np.geomspace(1e-4, 1, 20), np.linspace(1.0, 20, 40)])
    ell, sigma2 = 0.2, 1.0
    dist = x * ell
    got = h.matern(_cuda(dist), (sigma2, ell, nu, 0.0), precision=h.MIXED).cpu().numpy()
    want = matern.matern(dist, sigma2, ell, nu)
    err = np.abs(got - want) / np.maximum(want, 1e-12 * sigma2 / 2e-6)
    assert err.max() <= 2e-6, (nu, float(err.max()))


# --------------------------------------------------------- small cases -----
def _field(n, dim, theta, sub):
    rng = synth.rng_for(synth.W_TESTS, sub)
    pts = synth.uniform_points(n, dim, rng)
    w = synth.standard_normal(n, rng)
    z = dense.sample(pts, theta, w)
    return pts, z


@pytest.mark.parametrize("n", [1, 2, 7, 50, 64])
def test_single_leaf_exact(n):
    h = _h()
    theta = (1.3, 0.2, 0.9, 0.05)
    pts, z = _field(n, 2, theta, 400 + n)
    ref = dense.loglik(pts, z, theta)
    with h.Problem(_cuda(pts), leaf_size=64) as p:
        got = p.eval(theta, _cuda(z))
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-12 * max(1.0, abs(r)), (n, got, ref)


def _c1():
    rng = synth.rng_for(synth.W_SMALL_UNIFORM)
    pts = synth.uniform_points(2000, 2, rng)
    w = synth.standard_normal(2000, rng)
    theta = (1.0, 0.1, 0.5, 0.01)
    z = dense.sample(pts, theta, w)
    return pts, z, theta


def test_c1_parity_fp64():
    h = _h()
    pts, z, theta = _c1()
    ref = dense.loglik(pts, z, theta)
    with h.Problem(_cuda(pts), leaf_size=64, eta=2.0, aca_tol=1e-6) as p:
        got = p.eval(theta, _cuda(z))
        st = p.stats()
    print("C1 ref", ref, "got", got, "rel", _rel(got[0], ref[0]), st)
    assert _rel(got[0], ref[0]) <= 1e-6
    assert _rel(got[1], ref[1]) <= 1e-6


# nu -> the eps at which the n = 2000 configuration meets the 1e-6 target (the eps sweep measures it,
# tests/test_gpu_eps_sweep.py): smoother fields are worse conditioned and need a tighter eps
EPS_FOR_NU = {0.3: 1e-6, 1.0: 1e-6, 1.5: 1e-7, 2.5: 1e-8}


@pytest.mark.parametrize("nu", sorted(EPS_FOR_NU))
def test_c1_geometry_other_nu(nu):
    """Same points and data as the n=2000 case at other smoothness, at the eps
    that the sweep found to reach the small-n target: 1e-6 relative."""
    h = _h()
    pts, z, _ = _c1()
    theta = (1.0, 0.1, nu, 0.01)
    ref = dense.loglik(pts, z, theta)
    with h.Problem(_cuda(pts), leaf_size=64, eta=2.0, aca_tol=EPS_FOR_NU[nu], max_rank=64) as p:
        got = p.eval(theta, _cuda(z))
    print("nu", nu, "eps", EPS_FOR_NU[nu], "rel", _rel(got[0], ref[0]))
    assert _rel(got[0], ref[0]) <= 1e-6


@pytest.mark.parametrize("n,dim,leaf", [(129, 2, 64), (1000, 3, 32), (3001, 2, 100)])
def test_ragged_and_3d(n, dim, leaf):
    h = _h()
    theta = (0.8, 0.15, 0.7, 0.02)
    pts, z = _field(n, dim, theta, 500 + n)
    ref = dense.loglik(pts, z, theta)
    with h.Problem(_cuda(pts), leaf_size=leaf, aca_tol=1e-7) as p:
        got = p.eval(theta, _cuda(z))
    print(n, dim, "rel", _rel(got[0], ref[0]))
    assert _rel(got[0], ref[0]) <= 1e-6


def test_deterministic_repeat():
    h = _h()
    pts, z, theta = _c1()
    with h.Problem(_cuda(pts), leaf_size=64) as p:
        a = p.eval(theta, _cuda(z))
        b = p.eval(theta, _cuda(z))
    assert a == b


def test_not_spd_reported():
    h = _h()
    pts = np.array([[0.2, 0.2], [0.2, 0.2], [0.7, 0.1], [0.4, 0.9]])
    with h.Problem(_cuda(pts), leaf_size=64) as p:
        p.assemble((1.0, 0.3, 0.5, 0.0))
        with pytest.raises(h.NotSPD):
            p.factor()
        # recovers after a valid assemble
        got = p.eval((1.0, 0.3, 0.5, 0.1), _cuda(np.ones(4)))
    ref = dense.loglik(pts, np.ones(4), (1.0, 0.3, 0.5, 0.1))
    assert abs(got[0] - ref[0]) <= 1e-12 * abs(ref[0])


def test_state_machine_and_validation():
    h = _h()
    pts, z, theta = _c1()
    with h.Problem(_cuda(pts), leaf_size=64) as p:
        with pytest.raises(h.HmleError) as e:
            p.factor()
        assert e.value.status == h.HMLE_E_STATE
        with pytest.raises(h.HmleError) as e:
            p.loglik(_cuda(z))
        assert e.value.status == h.HMLE_E_STATE
        for bad in [(0.0, 0.1, 0.5, 0.01), (1.0, -1.0, 0.5, 0.01), (1.0, 0.1, 9.0, 0.01), (1.0, 0.1, 0.5, -1.0),
                    (float("nan"), 0.1, 0.5, 0.0)]:
            with pytest.raises(h.HmleError) as e:
                p.assemble(bad)
            assert e.value.status == h.HMLE_E_INVALID
        p.assemble(theta)
        p.factor()
        with pytest.raises(h.HmleError) as e:
            p.factor()
        assert e.value.status == h.HMLE_E_STATE


def test_sampler_matches_dense():
    """z = P^T L~ w at a tight accuracy equals the dense P^T chol(P C P^T) w, in
    norm and entry by entry."""
    h = _h()
    rng = synth.rng_for(synth.W_TESTS, 600)
    n = 1500
    pts = synth.uniform_points(n, 2, rng)
    w = synth.standard_normal(n, rng)
    theta = (1.0, 0.1, 1.0, 0.01)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-10, max_rank=64) as p:
        p.assemble(theta)
        p.factor()
        zg = p.sample(_cuda(w)).cpu().numpy()
        perm = p.export_tree()[0]
    C = dense.covariance(pts[perm], theta)
    y = dense.cholesky(C) @ w
    zr = np.empty(n)
    zr[perm] = y
    err = np.linalg.norm(zg - zr) / np.linalg.norm(zr)
    worst = np.abs(zg - zr).max() / np.abs(zr).max()
    print("sampler rel", err, "worst entry", worst)
    assert err <= 1e-7
    # element by element: every entry within 1e-7 of the field's largest entry
    assert worst <= 1e-7
