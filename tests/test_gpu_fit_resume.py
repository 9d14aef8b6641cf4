"""Checkpoint and resume of a real GPU fit (hmle_fit_resumable through the C
ABI): the Nelder-Mead search of Section 2 in the Section 5.1 coordinates on an
H-matrix problem (n = 1500, leaf 64, eps 1e-7) stopped after k iterations and
continued from its checkpoint, once or in several pieces, returns the
uninterrupted fit's estimate, log-likelihood and counts bit for bit (every
evaluation is a deterministic function of theta, so the continued search
visits the same points); both the four-parameter and the profiled search. A
checkpoint of the other search kind, of another problem size, of other data
or of another accuracy is refused (the checkpoint stores a fingerprint of the
data and the accuracy options)."""
import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _field(n=1500, seed=760):
    rng = synth.rng_for(synth.W_TESTS, seed)
    pts = synth.uniform_points(n, 2, rng)
    w = synth.standard_normal(n, rng)
    z = dense.sample(pts, (1.2, 0.1, 0.9, 0.02), w)
    return pts, z


def _same(a, b):
    assert a.theta == b.theta, (a.theta, b.theta)
    assert a.logL == b.logL, (a.logL, b.logL)
    assert (a.evals, a.iters, a.failed_evals, a.converged) == (b.evals, b.iters, b.failed_evals, b.converged)


@pytest.mark.parametrize("profile", [False, True])
def test_stopped_and_continued_fit_equals_uninterrupted(profile):
    import paper_2104_07146_amd as h
    pts, z = _field()
    dz = _cuda(z)
    print(f"fit resume profile={profile}", flush=True)
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-7) as p:
        full, _ = p.fit_resumable(dz, profile_variance=profile)
        assert full.converged
        # the plain entry point runs the same search
        _same(p.fit(dz, profile_variance=profile), full)
        # one stop after 7 iterations
        part, st = p.fit_resumable(dz, max_iter=7, profile_variance=profile)
        assert not part.converged and part.iters == 7
        rest, _ = p.fit_resumable(dz, state=st, profile_variance=profile)
        _same(rest, full)
        # several stops: 3, 10, 25 iterations, then to the end
        st = None
        for k in (3, 10, 25):
            part, st = p.fit_resumable(dz, state=st, max_iter=k, profile_variance=profile)
            assert part.iters == min(k, full.iters)
        rest, st_end = p.fit_resumable(dz, state=st, profile_variance=profile)
        _same(rest, full)
        # the final checkpoint evaluates nothing more
        again, _ = p.fit_resumable(dz, state=st_end, profile_variance=profile)
        _same(again, full)
        # the other search kind refuses the checkpoint
        with pytest.raises(Exception):
            p.fit_resumable(dz, state=st_end, profile_variance=not profile)
    print(f"  theta {full.theta} logL {full.logL:.6f} evals {full.evals} iters {full.iters}", flush=True)


def test_checkpoint_of_other_data_or_accuracy_is_refused():
    import paper_2104_07146_amd as h
    pts, z = _field()
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-6) as p:
        _, st = p.fit_resumable(_cuda(z), max_iter=2)
        z2 = z.copy()
        z2[17] += 1e-3
        with pytest.raises(Exception):
            p.fit_resumable(_cuda(z2), state=st)
        part, _ = p.fit_resumable(_cuda(z), state=st, max_iter=3)   # the same data continues
        assert part.iters == 3
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-7) as q:
        with pytest.raises(Exception):
            q.fit_resumable(_cuda(z), state=st)


def test_checkpoint_of_another_size_is_refused():
    import paper_2104_07146_amd as h
    pts, z = _field()
    with h.Problem(_cuda(pts), leaf_size=64, aca_tol=1e-6) as p:
        _, st = p.fit_resumable(_cuda(z), max_iter=2)
    pts2, z2 = _field(n=1400, seed=761)
    with h.Problem(_cuda(pts2), leaf_size=64, aca_tol=1e-6) as q:
        with pytest.raises(Exception):
            q.fit_resumable(_cuda(z2), state=st)
