"""The H-matrix-vector product (hmle_matvec) against the oracle, through the
C ABI: at n = 2000 (leaf 64, eps 1e-6) the GPU product equals the densified
exported H-matrix times x to rounding, and the exact covariance product to
the approximation accuracy; a batch acts block-diagonally; the call is only
valid between assembly and factorisation."""
import numpy as np
import pytest

import synth
from oracle import dense, densify

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _dense_of(p, n):
    perm, nodes, _, _ = p.export_tree()
    dense_ids, lr_ids = p.export_blocks()
    dA = []
    for i, (t, s) in enumerate(dense_ids):
        dA.append((int(nodes[t][0]), int(nodes[s][0]),
                   p.export_block(0, i, nodes[t][1] - nodes[t][0], nodes[s][1] - nodes[s][0])))
    lA = []
    for i, (t, s) in enumerate(lr_ids):
        U, V = p.export_block(1, i, nodes[t][1] - nodes[t][0], nodes[s][1] - nodes[s][0])
        lA.append((int(nodes[t][0]), int(nodes[s][0]), U, V))
    return perm, densify.densify_lower(n, dA, lA)


@pytest.mark.parametrize("nu,precision", [(0.5, 0), (1.5, 0), (1.0, 1)])
def test_matvec_matches_densified_and_exact(nu, precision):
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 700)
    n = 2000
    pts = synth.uniform_points(n, 2, rng)
    theta = (1.2, 0.1, nu, 0.01)
    x = rng.standard_normal((3, n))
    print(f"matvec nu={nu} precision={precision}", flush=True)
    with h.Problem(_cuda(pts), leaf_size=64, eta=2.0, aca_tol=1e-6, precision=precision) as p:
        p.assemble(theta)
        got = np.stack([p.matvec(_cuda(v)).cpu().numpy() for v in x])
        perm, Ct = _dense_of(p, n)
        again = p.matvec(_cuda(x[0])).cpu().numpy()
    np.testing.assert_array_equal(again, got[0])            # fixed summation order
    C = dense.covariance(pts, theta)
    inv = np.argsort(perm)
    for k in range(3):
        ref_h = (Ct @ x[k][perm])[inv]                        # the same H-matrix, densified on the host
        ref = C @ x[k]
        assert np.linalg.norm(got[k] - ref_h) <= 1e-12 * np.linalg.norm(ref_h)
        err = np.linalg.norm(got[k] - ref) / np.linalg.norm(ref)
        print(f"  probe {k}: ||C~x - Cx|| / ||Cx|| = {err:.2e}")
        assert err <= (1e-6 if precision == 0 else 1e-5)


def test_matvec_batch_is_block_diagonal():
    import torch
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 701)
    sizes = [700, 1300, 90]
    pts = [synth.uniform_points(m, 2, rng) for m in sizes]
    thetas = [(1.0, 0.1, 0.5, 0.02), (0.7, 0.2, 1.5, 0.01), (2.0, 0.05, 1.0, 0.1)]
    x = rng.standard_normal(sum(sizes))
    print("matvec batch", flush=True)
    with h.Batch([_cuda(a) for a in pts], leaf_size=64, eta=2.0, aca_tol=1e-8) as b:
        b.assemble(thetas)
        got = b.matvec(_cuda(x)).cpu().numpy()
    off = np.concatenate([[0], np.cumsum(sizes)])
    for q in range(3):
        ref = dense.covariance(pts[q], thetas[q]) @ x[off[q]:off[q + 1]]
        err = np.linalg.norm(got[off[q]:off[q + 1]] - ref) / np.linalg.norm(ref)
        assert err <= 1e-7, (q, err)


def test_matvec_state():
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 702)
    pts = synth.uniform_points(300, 2, rng)
    x = _cuda(rng.standard_normal(300))
    with h.Problem(_cuda(pts), leaf_size=32) as p:
        with pytest.raises(h.HmleError) as e:
            p.matvec(x)
        assert e.value.status == h.HMLE_E_STATE
        p.assemble((1.0, 0.1, 0.5, 0.01))
        p.matvec(x)
        p.factor()
        with pytest.raises(h.HmleError) as e:
            p.matvec(x)
        assert e.value.status == h.HMLE_E_STATE
