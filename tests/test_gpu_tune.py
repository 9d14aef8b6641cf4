"""GPU test of the schedule autotuner: it times every candidate of its grid
and returns one of them; the schedule options change only which workgroup
computes which products (so sums in another order and, at a threshold, a
truncation rank by one), so the log-likelihood with the chosen options agrees
with the default schedule far inside the H-approximation error."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_autotune_grid_and_agreement():
    import torch
    import paper_2104_07146_amd as h
    from oracle import dense
    rng = synth.rng_for(synth.W_TESTS, 700)
    n = 3000
    pts = synth.uniform_points(n, 2, rng)
    theta = (1.0, 0.1, 0.5, 0.01)
    z = dense.sample(pts, theta, synth.standard_normal(n, rng))
    dp = torch.tensor(pts, device="cuda")
    best, grid = h.autotune(dp, theta, leaf_size=64, aca_tol=1e-6)
    assert len(grid) == 9 and all(v > 0 for v in grid.values())
    assert (best["pair_chunk"], best["sketch_group"]) in grid
    assert grid[(best["pair_chunk"], best["sketch_group"])] == min(grid.values())
    zc = torch.tensor(z, device="cuda")
    with h.Problem(dp, leaf_size=64, aca_tol=1e-6) as p:
        a = p.eval(theta, zc)
    with h.Problem(dp, leaf_size=64, aca_tol=1e-6, **best) as p:
        b = p.eval(theta, zc)
    for pc, sg in [(4, 2), (2, 4)]:
        with h.Problem(dp, leaf_size=64, aca_tol=1e-6, pair_chunk=pc, sketch_group=sg) as p:
            c = p.eval(theta, zc)
        assert abs(c[0] - a[0]) <= 1e-8 * abs(a[0]), (pc, sg, c[0], a[0])
    assert abs(b[0] - a[0]) <= 1e-8 * abs(a[0])
    ref = dense.loglik(pts, z, theta)
    assert abs(b[0] - ref[0]) <= 1e-6 * abs(ref[0])
