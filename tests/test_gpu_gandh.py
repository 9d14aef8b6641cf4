"""The H-MLE on non-Gaussian data (Section 5, Test 2a): Tukey g-and-h fields
(eq. (8)) with the two parameter sets of the test, (xi, omega, g, h) =
(1, 2, 0.2, 0.2) and (1, 2, 0.5, 0.3), over a Gaussian field with Matern
(sigma^2, ell, nu, tau^2) = (1, 0.1, 1, 0) on uniform points.

The Gaussian model of eq. (1) has mean zero; the data are centred by their
sample mean before fitting (the location xi is not a covariance parameter).
The GPU fit (Nelder-Mead in the Section 5.1 coordinates, FP64 H path) is
compared with SciPy's Nelder-Mead on the dense oracle from the same start, by
the oracle's log-likelihood at the two optima (the likelihood of a misspecified
model is flat; theta is not compared), and the kriging predictions (eq. (4))
at held-out points with the GPU estimate against the oracle's predictions with
the same estimate; the RMSE (eq. (7)) against the held-out values is reported.
"""
import numpy as np
import pytest

import synth
from oracle import dense, krige, mle, reparam

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("xi,omega,g,hh", [(1.0, 2.0, 0.2, 0.2), (1.0, 2.0, 0.5, 0.3)])
def test_fit_on_tukey_g_and_h_field(xi, omega, g, hh):
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 730 + int(10 * g))
    n, m = 700, 100
    pts_all = synth.uniform_points(n + m, 2, rng)
    w = synth.standard_normal(n + m, rng)
    gauss = dense.sample(pts_all, (1.0, 0.1, 1.0, 0.0), w)
    t_all = synth.tukey_g_and_h(gauss, xi, omega, g, hh)
    pts, pts2 = pts_all[:n], pts_all[n:]
    mean = float(np.mean(t_all[:n]))
    z = t_all[:n] - mean
    z2 = t_all[n:] - mean
    v = float(np.var(z))
    start = (v, 0.12, 1.0, 0.05 * v)
    print(f"g-and-h ({xi}, {omega}, {g}, {hh}): oracle fit", flush=True)
    ref = mle.fit(pts, z, x0=reparam.from_theta(start), max_iter=400, tol=1e-4)
    print(f"  oracle theta {ref['theta']} logL {ref['logL']:.6f} evals {ref['nfev']}", flush=True)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-8) as p:
        fit = p.fit(_cuda(z), start=start, max_iter=400, tol=1e-4)
        p.assemble(fit.theta)
        p.factor()
        pred = p.predict(_cuda(z), _cuda(pts2)).cpu().numpy()
    l_gpu = dense.loglik(pts, z, fit.theta)[0]
    pred_ref = krige.predict(pts, z, pts2, fit.theta)
    rmse = krige.rmse(pred, z2)
    print(f"  gpu theta {fit.theta} logL(oracle) {l_gpu:.6f} evals {fit.evals}; RMSE {rmse:.4f} "
          f"(data sd {np.std(z2):.4f})", flush=True)
    assert fit.converged
    assert abs(l_gpu - ref["logL"]) <= 1e-4 * abs(ref["logL"])
    assert np.abs(pred - pred_ref).max() <= 1e-6 * max(1.0, np.abs(pred_ref).max())
    assert rmse < np.std(z2)
