"""What the trained start-proposal network gains over the method without it.

Held-out fields (n = 2000 uniform points, parameters from the training
ranges, data drawn by the H sampler at eps 1e-8; a seed stream the training
never used) are fitted by the same Nelder-Mead H-MLE three times: from the
paper's start (Section 5.1, with the nugget back-off), from the moment start
(sigma^2 = var Z, ell = 0.1, nu = 1, tau^2 = 0.05 var Z) and from the
network's proposal (trained weights shipped with the package). The optimiser
stays the arbiter: over the eight fields the learned start must need clearly
fewer evaluations than the paper's start (at most 0.6 times on average) and
no more than the moment start on average, and on every field it must end at
a likelihood at least as good as the better of the other two, up to the
optimiser's own resolution (simplex size 1e-4: 1e-2 absolute plus 1e-6
relative).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_learned_start_needs_fewer_evaluations():
    import torch
    import paper_2104_07146_amd as h
    from paper_2104_07146_amd import learned_start as ls
    net = ls.load()
    rng = synth.rng_for(synth.W_LEARNED, 8)
    ev = {"paper": [], "moment": [], "learned": []}
    for f in range(8):
        n = 2000
        pts = synth.uniform_points(n, 2, rng)
        th = synth.batch_theta(rng)
        w = synth.standard_normal(n, rng)
        dp = torch.tensor(pts, device="cuda")
        with h.Problem(dp, leaf_size=64, aca_tol=1e-8, max_rank=48) as ps:
            ps.assemble(th)
            ps.factor()
            z = ps.sample(torch.tensor(w, device="cuda"))
        v = float(torch.var(z))
        starts = {"paper": None, "moment": (v, 0.1, 1.0, 0.05 * v), "learned": ls.propose(net, dp, z)}
        res = {}
        with h.Problem(dp, leaf_size=64, aca_tol=1e-6) as p:
            for name, st in starts.items():
                res[name] = p.fit(z, start=st)
                ev[name].append(res[name].evals)
        print(f"field {f}: theta={tuple(round(x, 4) for x in th)} " +
              " ".join(f"{k}: evals {r.evals} logL {r.logL:.4f};" for k, r in res.items()), flush=True)
        best = max(res["paper"].logL, res["moment"].logL)
        assert res["learned"].logL >= best - 1e-2 - 1e-6 * abs(best), (f, {k: r.logL for k, r in res.items()})
    mean = {k: float(np.mean(v)) for k, v in ev.items()}
    print("mean evaluations", mean)
    assert mean["learned"] <= 0.6 * mean["paper"], mean
    assert mean["learned"] <= mean["moment"], mean
