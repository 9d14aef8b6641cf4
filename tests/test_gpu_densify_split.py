"""Densification split of the H error against the oracle (through the C ABI).

After hmle_assemble every block of the H-matrix C~ is exported and compared
with the exact block of the Matern covariance (eq. (2)): dense blocks entry by
entry, low-rank blocks by the cross-approximation bound of Section 2 (a fixed
accuracy eps per sub-block, read as ||A - U V^T||_F <= eps ||A||_F; the
partial-pivoting cross approximation is a heuristic, so the bar is 10 eps).
The densified C~ then splits the log-likelihood error into its two sources:
  approximation  |O1(C~) - O1(C)|   (the H-matrix itself),
  arithmetic     |L_gpu - O1(C~)|   (the H-Cholesky's truncated updates),
with O1 the dense float64 log-likelihood of eq. (1). After hmle_factor the
exported factor L~ is densified too:
  * 2 sum log diag(L~) is the GPU's log-determinant (the Section 2 identity)
    and equals slogdet(L~ L~^T) of the densified factor;
  * the GPU's quadratic form equals ||L~^{-1} P z||^2 by a dense triangular
    solve with the exported factor (so the GPU solve and reductions are exact
    for the factor they use);
  * ||L~ L~^T - C~||_F / ||C~||_F stays at the accuracy eps.
"""
import math

import numpy as np
import pytest
from scipy import linalg

import synth
from oracle import dense, densify

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _export(p, n, factored):
    """Blocks of the problem's current matrix in the internal order: dense
    (r0, c0, D) and low-rank (r0, c0, U, V)."""
    perm, nodes, _, _ = p.export_tree()
    dense_ids, lr_ids = p.export_blocks()
    dblocks, lblocks = [], []
    for i, (t, s) in enumerate(dense_ids):
        r0, r1, c0, c1 = nodes[t][0], nodes[t][1], nodes[s][0], nodes[s][1]
        D = p.export_block(0, i, r1 - r0, c1 - c0)
        if factored and t == s:
            D = np.tril(D)
        dblocks.append((int(r0), int(c0), D))
    for i, (t, s) in enumerate(lr_ids):
        r0, r1, c0, c1 = nodes[t][0], nodes[t][1], nodes[s][0], nodes[s][1]
        U, V = p.export_block(1, i, r1 - r0, c1 - c0)
        lblocks.append((int(r0), int(c0), U, V))
    return perm, dblocks, lblocks


CASES = {
    # (points, dim, leaf, eps, theta); the n = 2000 case is the small parity configuration
    "2d_n2000_nu0.5": (2000, 2, 64, 1e-6, (1.0, 0.1, 0.5, 0.01)),
    "2d_n2000_nu1.5": (2000, 2, 64, 1e-8, (1.0, 0.1, 1.5, 0.01)),
    "3d_n1500_nu1.0": (1500, 3, 64, 1e-6, (1.0, 0.15, 1.0, 0.01)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_densification_split(name):
    import paper_2104_07146_amd as h
    n, dim, leaf, eps, theta = CASES[name]
    rng = synth.rng_for(synth.W_SMALL_UNIFORM) if dim == 2 else synth.rng_for(synth.W_TESTS, 600)
    pts = synth.uniform_points(n, dim, rng)
    w = synth.standard_normal(n, rng)
    z = dense.sample(pts, theta, w)
    print(f"densify split {name}", flush=True)
    with h.Problem(_cuda(pts), leaf_size=leaf, eta=2.0, aca_tol=eps) as p:
        p.assemble(theta)
        perm, dA, lA = _export(p, n, factored=False)
        pp = pts[perm]
        # dense blocks: exact Matern entries (+ nugget on the diagonal)
        worst_dense = 0.0
        for r0, c0, D in dA:
            m, k = D.shape
            ref = dense.cross_covariance(pp[r0:r0 + m], pp[c0:c0 + k], theta)
            if r0 == c0:
                ref = ref + theta[3] * np.eye(m)
                D, ref = np.tril(D), np.tril(ref)
            worst_dense = max(worst_dense, float(np.abs(D - ref).max() / np.abs(ref).max()))
        assert worst_dense <= 1e-13, worst_dense
        # low-rank blocks: cross-approximation accuracy per block
        worst_lr, ranks = 0.0, []
        for r0, c0, U, V in lA:
            m, k = U.shape[0], V.shape[0]
            ref = dense.cross_covariance(pp[r0:r0 + m], pp[c0:c0 + k], theta)
            worst_lr = max(worst_lr, float(np.linalg.norm(ref - U @ V.T) / np.linalg.norm(ref)))
            ranks.append(U.shape[1])
        Ct = densify.densify_lower(n, dA, lA)
        p.factor()
        got = p.loglik(_cuda(z))
        _, dL, lL = _export(p, n, factored=True)
    L = densify.densify_lower(n, dL, lL, symmetric=False)
    zp = z[perm]
    exact = dense.loglik(pp, zp, theta)
    on_ct = dense.loglik_from_factor(dense.cholesky(Ct), zp)
    C = dense.covariance(pp, theta)
    approx = abs(on_ct[0] - exact[0]) / abs(exact[0])
    arith = abs(got[0] - on_ct[0]) / abs(exact[0])
    fact = float(np.linalg.norm(L @ L.T - Ct) / np.linalg.norm(Ct))
    block_err = float(np.linalg.norm(Ct - C) / np.linalg.norm(C))
    print(f"{name}: max rank {max(ranks)}, worst block {worst_lr:.2e} (eps {eps:.0e}), ||C~-C||/||C|| "
          f"{block_err:.2e}, ||LL^T-C~||/||C~|| {fact:.2e}; logL exact {exact[0]:.8f} on C~ {on_ct[0]:.8f} "
          f"gpu {got[0]:.8f}: approximation {approx:.2e}, arithmetic {arith:.2e}")
    assert worst_lr <= 10 * eps, worst_lr
    assert np.allclose(np.triu(L, 1), 0.0)
    diag = np.diag(L)
    assert (diag > 0).all()
    logdet_l = 2.0 * math.fsum(np.log(diag))
    assert abs(got[1] - logdet_l) <= 1e-12 * abs(logdet_l)
    sign, slog = np.linalg.slogdet(L @ L.T)
    assert sign > 0 and abs(slog - logdet_l) <= 1e-10 * abs(logdet_l)
    v = linalg.solve_triangular(L, zp, lower=True)
    assert abs(got[2] - float(v @ v)) <= 1e-10 * abs(got[2])
    assert fact <= 10 * eps, fact
    # the total error splits into its two parts and stays at the small-n target
    assert abs(got[0] - exact[0]) <= (approx + arith) * abs(exact[0]) * (1 + 1e-9) + 1e-9
    assert approx <= 1e-6 and arith <= 1e-6, (approx, arith)
