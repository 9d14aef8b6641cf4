"""Learned starting point for the maximum-likelihood fit.

The optimiser's cost depends on its start (Section 5.1; the conclusion
proposes precomputing the initial guess). This module trains the library's
start-proposal network (a fully connected tanh network, the family of
Section 4, trained with Adam as in Section 6) on fields the library itself
samples at known parameters, and proposes a start for new data:

  * training data: point sets of 4096 uniform points in the unit square,
    parameters drawn from the batched workload's ranges, fields drawn by the
    batched H-matrix sampler (hmle_sample on a batch), features by
    hmle_variogram, targets log(sigma2, range, nu, tau2);
  * training: hmle_mlp_fit_norm, then epochs of hmle_mlp_train_step over a
    seeded row order, a held-out validation share scored by hmle_mlp_grad;
  * proposal: features of (a seeded subset of 4096 points of) the data, then
    hmle_propose.

Every numerical step runs in the library's kernels; this file only moves
arrays and drives the loops. Run as a script:

  python -m paper_2104_07146_amd.learned_start train --fields 100000 --out FILE
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import Batch, Mlp, variogram

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "start_mlp.npz")
N_USED = 4096            # points a feature vector is computed from


def _synth():
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    return synth


def sample_training_set(n_fields: int, n_points: int = N_USED, group: int = 256, seed: int = 0,
                        eps: float = 1e-7, leaf: int = 64, log=print):
    """Features (rows x 33 float32, CUDA) and log-parameter targets (rows x 4
    float32, CUDA) of n_fields sampled fields. `group` point sets are built
    once as one batch; every round draws new parameters and noise for all of
    them. Problems whose factor is not positive definite are dropped."""
    import torch
    synth = _synth()
    rng = synth.rng_for(synth.W_LEARNED, 100 + seed)
    layouts = [torch.tensor(synth.uniform_points(n_points, 2, rng), device="cuda") for _ in range(group)]
    pts = torch.cat(layouts).contiguous()
    feats, targets = [], []
    have = 0
    t0 = time.perf_counter()
    with Batch(layouts, leaf_size=leaf, aca_tol=eps, max_rank=48) as b:
        rounds = 0
        while have < n_fields:
            thetas = [synth.batch_theta(rng) for _ in range(group)]
            b.assemble(thetas)
            ok = b.factor() == 0
            w = torch.tensor(synth.standard_normal(group * n_points, rng), device="cuda")
            z = b.sample(w)
            f = variogram(pts, z, b.offsets)
            keep = torch.tensor(np.flatnonzero(ok), device="cuda")
            lt = torch.tensor(np.log(np.array(thetas, dtype=np.float64)), dtype=torch.float32, device="cuda")
            feats.append(f.index_select(0, keep))
            targets.append(lt.index_select(0, keep))
            have += int(ok.sum())
            rounds += 1
            if rounds % 20 == 0 or have >= n_fields:
                log(f"# sampled {have} fields in {rounds} rounds, {time.perf_counter() - t0:.1f} s")
    x = torch.cat(feats)[:n_fields].contiguous()
    y = torch.cat(targets)[:n_fields].contiguous()
    return x, y


def train(x, lt, epochs: int = 50, batch: int = 1024, lr: float = 1e-3, val_frac: float = 0.05, seed: int = 0,
          log=print):
    """Train a fresh network on (x, lt); returns (Mlp, report dict)."""
    import torch
    synth = _synth()
    rng = synth.rng_for(synth.W_LEARNED, 200 + seed)
    n = int(x.shape[0])
    order = torch.tensor(synth.minibatch_order(n, rng), device=x.device, dtype=torch.long)
    n_val = max(1, int(round(val_frac * n)))
    val, tr = order[:n_val], order[n_val:]
    xv, lv = x.index_select(0, val).contiguous(), lt.index_select(0, val).contiguous()
    xt, lt_t = x.index_select(0, tr).contiguous(), lt.index_select(0, tr).contiguous()
    net = Mlp(synth.mlp_init(rng))
    net.fit_norm(xt, lt_t)
    nt = int(xt.shape[0])
    history = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.tensor(synth.minibatch_order(nt, rng), device=x.device)
        for s in range(0, nt, batch):
            idx = perm[s:s + batch].contiguous()
            net.train_step(xt, lt_t, idx, lr=lr, want_loss=False)
        val_mse = net.grad(xv, lv)[1]
        history.append(val_mse)
        if ep % 5 == 4 or ep == epochs - 1:
            log(f"# epoch {ep + 1}: validation mse {val_mse:.4f} ({time.perf_counter() - t0:.1f} s)")
    steps = epochs * math.ceil(nt / batch)
    return net, {"fields": n, "train": nt, "val": int(n_val), "epochs": epochs, "batch": batch, "lr": lr,
                 "val_mse": history[-1], "val_mse_first": history[0], "steps": steps,
                 "train_s": time.perf_counter() - t0}


def save(net: Mlp, path: str, report: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.params(), norm=net.norm(), report=np.array(json.dumps(report)))


def load(path: str = DEFAULT_WEIGHTS) -> Mlp:
    d = np.load(path, allow_pickle=False)
    net = Mlp(d["params"])
    net.set_norm(d["norm"])
    return net


def features_of(pts, z, seed: int = 0):
    """Features (1 x 33, CUDA) of one field from a seeded subset of at most
    4096 of its points."""
    import torch
    synth = _synth()
    n = int(pts.shape[0])
    sel = synth.subset_indices(n, N_USED, synth.rng_for(synth.W_LEARNED, 300 + seed))
    return variogram(pts, z, np.array([0, n]), torch.tensor(sel, device=pts.device),
                     np.array([0, len(sel)]))


def propose(net: Mlp, pts, z, seed: int = 0):
    """Start (sigma2, range, nu, tau2) for data z at points pts (CUDA float64)."""
    return net.propose(features_of(pts, z, seed)[0])


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--fields", type=int, default=100000)
    t.add_argument("--group", type=int, default=256)
    t.add_argument("--epochs", type=int, default=50)
    t.add_argument("--eps", type=float, default=1e-7)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    a = ap.parse_args(argv)
    if a.cmd == "train":
        t0 = time.perf_counter()
        x, lt = sample_training_set(a.fields, group=a.group, eps=a.eps, log=lambda s: print(s, flush=True))
        t_sample = time.perf_counter() - t0
        net, rep = train(x, lt, epochs=a.epochs, log=lambda s: print(s, flush=True))
        rep["sample_s"] = t_sample
        rep["sampler_eps"] = a.eps
        save(net, a.out, rep)
        print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
