"""Accuracy sweep at the small parity configuration (n = 2000 uniform points,
leaf 64, eta 2, nugget 0.01): the relative log-likelihood error against the
dense oracle (eq. (1)) for each smoothness over eps in {1e-6 ... 1e-9}. The
error must fall to the small-n target 1e-6 at the eps gated here per nu (the
largest eps of the sweep that meets it, measured), and every tighter eps must
meet it too."""
import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu

EPS = [1e-6, 1e-7, 1e-8, 1e-9]
# nu -> the eps at which the 1e-6 target is met on this configuration
# (measured at eps 1e-6: 6.5e-9, 3.6e-9, 2.4e-7 for nu 0.3, 0.5, 1; nu 1.5: 3.4e-6 at 1e-6, 2.4e-7 at 1e-7)
GATE = {0.3: 1e-6, 0.5: 1e-6, 1.0: 1e-6, 1.5: 1e-7, 2.5: 1e-8}


@pytest.mark.parametrize("nu", sorted(GATE))
def test_eps_sweep_reaches_target(nu):
    import torch
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_SMALL_UNIFORM)
    pts = synth.uniform_points(2000, 2, rng)
    w = synth.standard_normal(2000, rng)
    z0 = dense.sample(pts, (1.0, 0.1, 0.5, 0.01), w)
    theta = (1.0, 0.1, nu, 0.01)
    ref = dense.loglik(pts, z0, theta)[0]
    dpts, dz = torch.tensor(pts, device="cuda"), torch.tensor(z0, device="cuda")
    errs = {}
    for eps in EPS:
        with h.Problem(dpts, leaf_size=64, eta=2.0, aca_tol=eps, max_rank=64) as p:
            got = p.eval(theta, dz)[0]
            st = p.stats()
        errs[eps] = abs(got - ref) / abs(ref)
        print(f"nu={nu} eps={eps:.0e}: rel err {errs[eps]:.2e} (rank max {st['rank_max']}, cap hits "
              f"{st['cap_hits']})", flush=True)
    for eps in EPS:
        if eps <= GATE[nu]:
            assert errs[eps] <= 1e-6, (nu, eps, errs[eps])
