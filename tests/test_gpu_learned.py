"""GPU parity of the learned-start kernels against the float64 oracle.

Tolerances: variogram features (float64 sums, float32 output) 1e-6 relative
(absolute below 1); network outputs 1e-4 (float32 arithmetic); gradients
1e-3 relative in norm and per component above 1e-3 of the largest (float32 vs
float64); Adam updates to 1% of a step where the gradient is not tiny.
"""
import numpy as np
import pytest

import synth
from oracle import learned

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a, dtype=np.float64):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _close_feat(got, want):
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    return float(err.max())


@pytest.mark.parametrize("dim", [2, 3])
def test_variogram_matches_oracle(dim):
    h = _h()
    rng = synth.rng_for(synth.W_LEARNED, 10 + dim)
    sizes = [1, 2, 127, 128, 129, 300, 1000]
    pts = [rng.random((n, dim)) for n in sizes]
    zs = [rng.standard_normal(n) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    print(f"variogram dim={dim} sizes={sizes}", flush=True)
    got = h.variogram(_cuda(np.concatenate(pts)), _cuda(np.concatenate(zs)), off).cpu().numpy()
    for q in range(len(sizes)):
        want = learned.variogram_features(pts[q], zs[q])
        assert _close_feat(got[q], want) <= 1e-6, (q, sizes[q])
    again = h.variogram(_cuda(np.concatenate(pts)), _cuda(np.concatenate(zs)), off).cpu().numpy()
    np.testing.assert_array_equal(got, again)


def test_variogram_subset_of_a_large_field():
    h = _h()
    rng = synth.rng_for(synth.W_LEARNED, 20)
    sizes = [20000, 5000]
    pts = [rng.random((n, 2)) for n in sizes]
    zs = [rng.standard_normal(n) for n in sizes]
    sel = [synth.subset_indices(n, 4096, rng) for n in sizes]
    off = np.array([0, sizes[0], sum(sizes)], dtype=np.int64)
    soff = np.array([0, 4096, 8192], dtype=np.int64)
    got = h.variogram(_cuda(np.concatenate(pts)), _cuda(np.concatenate(zs)), off,
                      _cuda(np.concatenate(sel), np.int32), soff).cpu().numpy()
    for q in range(2):
        want = learned.variogram_features(pts[q], zs[q], sel[q])
        assert _close_feat(got[q], want) <= 1e-6
        assert abs(got[q, 32] - np.log(4096)) < 1e-6


def test_variogram_rejects_bad_subset():
    h = _h()
    pts = _cuda(np.random.default_rng(0).random((10, 2)))
    z = _cuda(np.zeros(10))
    with pytest.raises(h.HmleError):
        h.variogram(pts, z, np.array([0, 10]), _cuda(np.array([0, 10]), np.int32), np.array([0, 2]))


def _net(seed):
    h = _h()
    rng = synth.rng_for(synth.W_LEARNED, seed)
    params = synth.mlp_init(rng)
    X = rng.standard_normal((300, 33)).astype(np.float32) * 2 + 1
    LT = rng.standard_normal((300, 4)).astype(np.float32) - 1
    mu_x, sd_x = learned.norm_stats(X)
    mu_y, sd_y = learned.norm_stats(LT)
    norm = np.concatenate([mu_x, sd_x, mu_y, sd_y]).astype(np.float32)
    return h, rng, params, X, LT, norm


def test_network_forward_matches_oracle():
    h, rng, params, X, LT, norm = _net(30)
    with h.Mlp(params) as net:
        net.set_norm(norm)
        y = net.forward(_cuda(X, np.float32)).cpu().numpy()
        np.testing.assert_array_equal(net.params(), params)
    n32 = norm.astype(np.float64)
    xs = learned.standardise(X.astype(np.float64), n32[:33], n32[33:66])
    _, ys = learned.forward(params.astype(np.float64), xs)
    want = ys * n32[70:74] + n32[66:70]
    err = np.abs(y - want) / np.maximum(1.0, np.abs(want))
    assert err.max() <= 1e-4, float(err.max())


def _ref_grad(params, X, LT, norm, rows):
    n = norm.astype(np.float64)
    xs = learned.standardise(X[rows].astype(np.float64), n[:33], n[33:66])
    ts = learned.standardise(LT[rows].astype(np.float64), n[66:70], n[70:74])
    return learned.loss_and_grad(params.astype(np.float64), xs, ts)


def test_network_gradient_matches_oracle():
    import torch
    h, rng, params, X, LT, norm = _net(40)
    idx = rng.permutation(300)[:237].astype(np.int32)     # a ragged batch through a row list
    with h.Mlp(params) as net:
        net.set_norm(norm)
        g, loss = net.grad(_cuda(X, np.float32), _cuda(LT, np.float32), _cuda(idx, np.int32))
        g = g.cpu().numpy()
        g_all, loss_all = net.grad(_cuda(X, np.float32), _cuda(LT, np.float32))
    L, ref = _ref_grad(params, X, LT, norm, idx)
    assert abs(loss - L) <= 1e-5 * L
    assert np.linalg.norm(g - ref) <= 1e-3 * np.linalg.norm(ref)
    big = np.abs(ref) > 1e-3 * np.abs(ref).max()
    assert (np.abs(g - ref)[big] / np.abs(ref)[big]).max() <= 1e-3
    L2, ref2 = _ref_grad(params, X, LT, norm, np.arange(300))
    assert abs(loss_all - L2) <= 1e-5 * L2
    assert np.linalg.norm(g_all.cpu().numpy() - ref2) <= 1e-3 * np.linalg.norm(ref2)


def test_adam_steps_match_oracle():
    h, rng, params, X, LT, norm = _net(50)
    lr = 1e-3
    p = params.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    batches = [rng.permutation(300)[:128].astype(np.int32) for _ in range(3)]
    with h.Mlp(params) as net:
        net.set_norm(norm)
        for t, idx in enumerate(batches, start=1):
            net.train_step(_cuda(X, np.float32), _cuda(LT, np.float32), _cuda(idx, np.int32), lr=lr)
            _, g = _ref_grad(p, X, LT, norm, idx)
            p, m, v = learned.adam_step(p, g, m, v, t, lr)
        got = net.params().astype(np.float64)
    # components whose gradients are tiny may take either sign in float32
    _, g0 = _ref_grad(params, X, LT, norm, batches[0])
    sure = np.abs(g0) > 1e-3 * np.abs(g0).max()
    assert np.abs(got - p)[sure].max() <= 0.01 * lr * 3
    assert np.abs(got - p).max() <= 2 * lr * 3


def test_fit_norm_matches_oracle():
    h, rng, params, X, LT, norm = _net(60)
    with h.Mlp(params) as net:
        net.fit_norm(_cuda(X, np.float32), _cuda(LT, np.float32))
        got = net.norm()
    mu_x, sd_x = learned.norm_stats(X, flat=1e30)
    mu_y, sd_y = learned.norm_stats(LT)
    want = np.concatenate([mu_x, sd_x, mu_y, sd_y])
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-6)
    # a constant feature column is switched off
    Xc = X.copy()
    Xc[:, 32] = 8.3
    with h.Mlp(params) as net:
        net.fit_norm(_cuda(Xc, np.float32), _cuda(LT, np.float32))
        assert net.norm()[33 + 32] == np.float32(1e30)


def test_training_reduces_loss_and_propose_is_consistent():
    """Targets that are a smooth function of the inputs: 300 Adam steps on the
    device cut the loss by half or more; the proposal is exp of the forward pass."""
    h, rng, params, X, _, _ = _net(70)
    W = rng.standard_normal((33, 4)) * 0.3
    LT = np.tanh(X @ W * 0.2).astype(np.float32) * 2 - 1
    xc, lc = _cuda(X, np.float32), _cuda(LT, np.float32)
    with h.Mlp(params) as net:
        net.fit_norm(xc, lc)
        first = net.grad(xc, lc)[1]
        for step in range(300):
            idx = _cuda(synth.minibatch_order(300, rng)[:100], np.int32)
            net.train_step(xc, lc, idx, lr=3e-3, want_loss=False)
        last = net.grad(xc, lc)[1]
        assert last <= 0.5 * first, (first, last)
        y = net.forward(xc[:1]).cpu().numpy()[0]
        th = net.propose(xc[0])
    box = [(1e-6, 1e6), (1e-4, 10.0), (0.05, 8.0), (1e-10, 1e3)]
    for k in range(4):
        assert abs(th[k] - float(np.clip(np.exp(y[k]), *box[k]))) <= 1e-6 * th[k]
