"""GPU tests of kriging prediction (hmle_predict, eq. (4)) against the dense
oracle: the H path solves with the H-factor (forward and backward
substitution) and applies the cross-covariance exactly, so at a tight
approximation accuracy it must agree with C21 C11^{-1} Z1 to the accuracy of
the factor. Sizes are ragged (training points not a multiple of the leaf,
new points not a multiple of the kernel's point tile); a batch and a problem
that is not factored are refused.
"""
import numpy as np
import pytest

import synth
from oracle import dense, krige

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("nu,precision", [(0.5, "fp64"), (1.5, "fp64"), (0.5, "mixed")])
def test_predict_matches_oracle(nu, precision):
    h = _h()
    rng = synth.rng_for(synth.W_TESTS, 940)
    pts = synth.uniform_points(1999, 2, rng)
    new = synth.uniform_points(301, 2, rng)
    theta = (1.2, 0.1, nu, 0.01)
    z = dense.sample(pts, theta, synth.standard_normal(len(pts), rng))
    ref = krige.predict(pts, z, new, theta)
    prec = h.MIXED if precision == "mixed" else h.FP64
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8, precision=prec) as p:
        p.assemble(theta)
        p.factor()
        got = p.predict(_cuda(z), _cuda(new)).cpu().numpy()
        again = p.predict(_cuda(z), _cuda(new)).cpu().numpy()
        empty = p.predict(_cuda(z), _cuda(np.zeros((0, 2))))
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("nu", nu, precision, "max rel err", err)
    assert np.array_equal(got, again)          # deterministic
    assert empty.numel() == 0
    assert err <= (2e-3 if precision == "mixed" else 1e-6)


def test_predict_refuses_batch_and_unfactored():
    h = _h()
    rng = synth.rng_for(synth.W_TESTS, 941)
    pts = synth.uniform_points(300, 2, rng)
    z = synth.standard_normal(300, rng)
    new = _cuda(synth.uniform_points(5, 2, rng))
    with h.Problem(_cuda(pts), leaf_size=64) as p:
        with pytest.raises(h.HmleError):
            p.predict(_cuda(z), new)
    with h.Batch([_cuda(pts), _cuda(pts)], leaf_size=64) as b:
        b.assemble([(1.0, 0.1, 0.5, 0.01)] * 2)
        b.factor()
        with pytest.raises(h.HmleError):
            import ctypes
            import torch
            out = torch.empty(5, dtype=torch.float64, device="cuda")
            zz = _cuda(np.concatenate([z, z]))
            h._check(h.lib().hmle_predict(b._h, h._ptr(zz), h._ptr(new), 5, h._ptr(out)), b._h)


@pytest.mark.parametrize("nu,precision", [(0.5, "fp64"), (1.5, "fp64"), (0.5, "mixed")])
def test_predict_var_matches_oracle(nu, precision):
    h = _h()
    rng = synth.rng_for(synth.W_TESTS, 942)
    pts = synth.uniform_points(1999, 2, rng)
    new = synth.uniform_points(61, 2, rng)
    theta = (1.2, 0.1, nu, 0.01)
    ref = krige.variance(pts, new, theta)
    prec = h.MIXED if precision == "mixed" else h.FP64
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8, precision=prec) as p:
        p.assemble(theta)
        p.factor()
        got = p.predict_var(_cuda(new)).cpu().numpy()
        empty = p.predict_var(_cuda(np.zeros((0, 2))))
    err = np.max(np.abs(got - ref)) / theta[0]
    print("variance nu", nu, precision, "max err / sigma2", err, "range", ref.min(), ref.max())
    assert empty.numel() == 0
    assert err <= (1e-3 if precision == "mixed" else 1e-6)
