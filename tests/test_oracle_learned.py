"""Pins of the learned-start oracle (variogram features, network, Adam)
against brute force, a hand-worked example, exact boundaries, finite
differences and invariants of Adam. CPU only."""
import math
import os

import numpy as np
import pytest

import synth
from oracle import learned

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _brute_sums(pts, z):
    m, dim = pts.shape
    sums = [0.0] * 32
    counts = [0] * 32
    for i in range(m):
        for j in range(i + 1, m):
            h = math.sqrt(sum((pts[i, k] - pts[j, k]) ** 2 for k in range(dim)))
            b = math.floor(64 * h)
            if b < 32:
                sums[b] += (z[i] - z[j]) ** 2
                counts[b] += 1
    return np.array(sums), np.array(counts)


@pytest.mark.parametrize("dim", [2, 3])
def test_variogram_matches_brute_force(dim):
    rng = synth.rng_for(synth.W_TESTS, 500 + dim)
    pts = rng.random((60, dim)) * 0.6
    z = rng.standard_normal(60)
    s, c = learned.variogram_sums(pts, z)
    bs, bc = _brute_sums(pts, z)
    np.testing.assert_array_equal(c, bc)
    np.testing.assert_allclose(s, bs, rtol=1e-13, atol=0)
    f = learned.variogram_features(pts, z)
    nz = bc > 0
    np.testing.assert_allclose(f[:32][nz], np.log(bs[nz] / (2 * bc[nz])), rtol=1e-13)
    assert (f[:32][~nz] == 0).all()
    assert f[32] == math.log(60)


def test_variogram_golden_example():
    vals = {}
    for line in open(os.path.join(GOLDEN, "variogram_4pts.txt")):
        if line.startswith("#") or not line.strip():
            continue
        key, *nums = line.split()
        vals[key] = np.array([float(v) for v in nums])
    pts = vals["points"].reshape(-1, 2)
    f = learned.variogram_features(pts, vals["z"])
    np.testing.assert_allclose(f[:4], np.log(vals["gamma"]), rtol=1e-15)
    assert (f[4:32] == 0).all()
    assert f[32] == math.log(4)


def test_pair_bins_exact_boundaries():
    k = np.arange(1, 33)
    h2 = (k / 64.0) ** 2                 # exact in binary
    got = learned.pair_bins(h2)
    np.testing.assert_array_equal(got, np.where(k < 32, k, -1))
    below = np.nextafter(h2, 0)
    np.testing.assert_array_equal(learned.pair_bins(below), k - 1)
    assert learned.pair_bins(np.array([0.0]))[0] == 0


def test_variogram_subset_and_permutation():
    rng = synth.rng_for(synth.W_TESTS, 510)
    pts = rng.random((200, 2))
    z = rng.standard_normal(200)
    idx = np.sort(rng.choice(200, 70, replace=False))
    np.testing.assert_array_equal(learned.variogram_features(pts, z, idx), learned.variogram_features(pts[idx], z[idx]))
    p = rng.permutation(200)
    np.testing.assert_allclose(learned.variogram_features(pts[p], z[p]), learned.variogram_features(pts, z),
                               rtol=1e-12)
    # a constant field: every bin's gamma is 0 -> the floor
    f = learned.variogram_features(pts, np.full(200, 3.0))
    filled = learned.variogram_sums(pts, z)[1] > 0
    np.testing.assert_array_equal(f[:32][filled], np.log(1e-30))


def _params(seed, scale=0.3):
    rng = synth.rng_for(synth.W_TESTS, seed)
    return rng.standard_normal(learned.n_params()) * scale


def _brute_forward(params, x):
    layers = learned.unpack(params)
    a = list(x)
    for li, (W, b) in enumerate(layers):
        out = []
        for o in range(W.shape[0]):
            s = b[o]
            for i in range(W.shape[1]):
                s += W[o, i] * a[i]
            out.append(math.tanh(s) if li < len(layers) - 1 else s)
        a = out
    return np.array(a)


def test_network_shape_and_forward_brute_force():
    assert learned.n_params() == 33 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 4 + 4 == 37892
    p = _params(520, 0.1)
    X = synth.rng_for(synth.W_TESTS, 521).standard_normal((2, 33))
    _, Y = learned.forward(p, X)
    for r in range(2):
        np.testing.assert_allclose(Y[r], _brute_forward(p, X[r]), rtol=1e-12, atol=1e-14)


def _fd_check(loss_and_grad, loss_fn, p, X, T, idx, h=1e-5):
    _, g = loss_and_grad(p, X, T)
    num = np.empty(len(idx))
    for k, i in enumerate(idx):
        e = np.zeros_like(p)
        e[i] = h
        num[k] = (loss_fn(p + e, X, T) - loss_fn(p - e, X, T)) / (2 * h)
    # relative error, with a floor of 1e-6 of the largest component (the central
    # difference itself carries about 1e-10 of absolute rounding error)
    return np.max(np.abs(num - g[idx]) / (np.abs(num) + 1e-6 * np.abs(num).max()))


def _fd_indices(rng):
    # every layer's weights and biases
    idx, off = [], 0
    for i, o in learned.LAYERS:
        idx += list(off + rng.choice(i * o, 40, replace=False))
        off += i * o
        idx += list(off + rng.choice(o, min(o, 8), replace=False))
        off += o
    return np.array(idx)


def test_gradient_matches_finite_differences():
    rng = synth.rng_for(synth.W_TESTS, 530)
    p = _params(531, 0.2)
    X = rng.standard_normal((5, 33))
    T = rng.standard_normal((5, 4))
    err = _fd_check(learned.loss_and_grad, learned.loss, p, X, T, _fd_indices(rng))
    assert err <= 1e-5, err


def test_gradient_check_catches_a_wrong_tanh_derivative():
    """A plausible slip (d tanh = 1 - tanh instead of 1 - tanh^2) fails the check."""
    def bad(params, X, T):
        layers = learned.unpack(params)
        acts, Y = learned.forward(params, X)
        B, K = Y.shape
        dA = 2.0 * (Y - T) / (B * K)
        grads = []
        for li in range(len(layers) - 1, -1, -1):
            W, _ = layers[li]
            grads.append((dA.T @ acts[li], dA.sum(axis=0)))
            if li > 0:
                dA = (dA @ W) * (1.0 - acts[li])
        grads.reverse()
        return 0.0, np.concatenate([np.concatenate([a.ravel(), b]) for a, b in grads])
    rng = synth.rng_for(synth.W_TESTS, 540)
    p = _params(541, 0.2)
    X = rng.standard_normal((5, 33))
    T = rng.standard_normal((5, 4))
    assert _fd_check(bad, learned.loss, p, X, T, _fd_indices(rng)) > 1e-2


def test_adam_constant_gradient_moves_by_lr_per_step():
    """With the same gradient every step the bias-corrected moments equal g and
    g^2 exactly, so every step moves each parameter by lr * g / (|g| + eps)."""
    rng = synth.rng_for(synth.W_TESTS, 550)
    g = rng.standard_normal(1000) * np.logspace(-3, 3, 1000)
    p0 = rng.standard_normal(1000)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    lr = 1e-3
    for t in range(1, 51):
        p, m, v = learned.adam_step(p, g, m, v, t, lr)
    np.testing.assert_allclose(p, p0 - 50 * lr * g / (np.abs(g) + learned.ADAM_EPS), rtol=0, atol=1e-12)


def test_adam_is_invariant_to_gradient_scale():
    rng = synth.rng_for(synth.W_TESTS, 560)
    p0 = rng.standard_normal(100)
    # components bounded away from 0, where eps = 1e-8 is negligible
    gs = [np.sign(rng.standard_normal(100)) * (0.5 + np.abs(rng.standard_normal(100))) for _ in range(5)]
    outs = []
    for c in (1.0, 1000.0):
        p, m, v = p0.copy(), np.zeros(100), np.zeros(100)
        for t, g in enumerate(gs, start=1):
            p, m, v = learned.adam_step(p, c * g, m, v, t, 1e-2)
        outs.append(p)
    np.testing.assert_allclose(outs[0], outs[1], rtol=0, atol=1e-8)


def test_norm_stats():
    a = np.array([[1.0, 5.0], [3.0, 5.0]])
    mu, sd = learned.norm_stats(a)
    np.testing.assert_array_equal(mu, [2.0, 5.0])
    np.testing.assert_array_equal(sd, [1.0, 1e-6])
    _, sd = learned.norm_stats(a, flat=1e30)
    np.testing.assert_array_equal(sd, [1.0, 1e30])
