"""GPU tests of the candidate-batched fit (hmle_fit_batch).

The batched fit runs the Nelder-Mead iteration of hmle_fit and evaluates the
points an iteration may need together on copies of one point set. Batched
values equal single ones bit for bit, so the estimate, the log-likelihood and
the evaluation, iteration and failure counts must equal those of hmle_fit on
one copy exactly; only the number of batched rounds is smaller. A batch whose
problems are not copies of one point set is refused.
"""
import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _field(n, theta, sub):
    rng = synth.rng_for(synth.W_TESTS, sub)
    pts = synth.uniform_points(n, 2, rng)
    w = synth.standard_normal(n, rng)
    return pts, dense.sample(pts, theta, w)


@pytest.mark.parametrize("count,start", [(4, "moment"), (2, "moment"), (3, None)])
def test_batched_fit_equals_sequential(count, start):
    h = _h()
    pts, z = _field(900, (1.0, 0.1, 0.7, 0.02), 810 + count)
    st = None if start is None else (float(np.var(z)), 0.12, 1.0, 0.05 * float(np.var(z)))
    opts = dict(leaf_size=64, aca_tol=1e-7)
    kw = dict(start=st, max_iter=400 if start else 60, tol=1e-4)
    dp, dz = _cuda(pts), _cuda(z)
    with h.Problem(dp, **opts) as p:
        seq = p.fit(dz, **kw)
    with h.Batch([dp] * count, **opts) as b:
        bat, rounds = b.fit(dz, **kw)
    print("sequential", seq, "batched", bat, "rounds", rounds)
    assert bat.status == seq.status
    assert bat.theta == seq.theta
    assert bat.logL == seq.logL
    assert (bat.evals, bat.iters, bat.failed_evals, bat.converged) == (seq.evals, seq.iters, seq.failed_evals,
                                                                         seq.converged)
    assert 0 < rounds < bat.evals
    if count >= 4:
        # every iteration needs one round, a shrink one more
        assert rounds <= bat.iters + 2 + (bat.evals - bat.iters) // 4 + 31


def test_batched_fit_refuses_different_point_sets():
    h = _h()
    pts, z = _field(300, (1.0, 0.1, 0.5, 0.02), 820)
    other = pts.copy()
    other[0, 0] += 1e-3
    with h.Batch([_cuda(pts), _cuda(other)], leaf_size=64, aca_tol=1e-6) as b:
        with pytest.raises(h.HmleError):
            b.fit(_cuda(z), max_iter=5)
    with h.Batch([_cuda(pts), _cuda(pts[:299])], leaf_size=64, aca_tol=1e-6) as b:
        with pytest.raises(h.HmleError):
            b.fit(_cuda(z), max_iter=5)
