"""Learned starting point: variogram features of a field and the fully
connected network that maps them to a start for the optimiser.
TEST INFRASTRUCTURE ONLY (see the package header): plain NumPy, float64.

The paper's deep-learning baseline (Section 4) is a fully connected network:
every layer a matrix-vector product with the connection weights followed by a
non-linear activation, trained by gradient descent; Section 6 reports tanh
activations and the Adam optimizer. The conclusion names precomputing the
optimiser's initial guess as the remedy for long fits (Section 5.1's start
can need hundreds of iterations). Here such a network proposes the start.

Readings (the paper fixes none of these):
  * Features (33): for the pairs i < j of the points used, with pair
    distance h, bin b = floor(64 h) for h < 1/2 (32 bins of width 1/64);
    gamma_b = sum over the bin's pairs of (z_i - z_j)^2 / (2 count_b);
    feature b = log(max(gamma_b, 1e-30)), and 0 for an empty bin;
    feature 32 = log(number of points used).
  * The bin is decided from h^2 = dx^2 + dy^2 (+ dz^2), each product and sum
    rounded on its own (no fused multiply-add): b = the largest integer k
    with k^2 <= 4096 h^2, so no square root is involved.
  * Points used: all, or a subset the caller passes (index list).
  * Standardisation: column means and deviations of the training data; a
    feature whose deviation is below 1e-6 is switched off (scale 1e30), a
    target's deviation is floored at 1e-6.
  * Network: 33 -> 128 -> 128 -> 128 -> 4, tanh on the three hidden layers,
    linear output, each layer y = x W^T + b (W: out x in, row-major). Inputs
    are standardised (x - mu_x) / sd_x, targets are standardised log theta
    t = (log theta - mu_y) / sd_y; loss = mean over rows and outputs of
    (y - t)^2.
  * Flat parameter order: W1, b1, W2, b2, W3, b3, W4, b4.
  * Adam (Kingma and Ba, 2015): beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
    bias-corrected moments, step t counted from 1.
"""
from __future__ import annotations

import numpy as np

N_BINS = 32
N_FEAT = N_BINS + 1
LAYERS = [(33, 128), (128, 128), (128, 128), (128, 4)]   # (in, out)
BETA1, BETA2, ADAM_EPS = 0.9, 0.999, 1e-8


def n_params() -> int:
    return sum(i * o + o for i, o in LAYERS)


# ------------------------------------------------------------ features -----
def pair_bins(h2: np.ndarray) -> np.ndarray:
    """Largest k with k^2 <= 4096 h2 (= floor(64 sqrt(h2))), exactly; -1 for
    pairs at distance >= 1/2 (k >= 32)."""
    s = 4096.0 * h2                          # exact: power-of-two scaling
    b = np.floor(np.sqrt(s)).astype(np.int64)
    b = np.where((b + 1).astype(np.float64) ** 2 <= s, b + 1, b)
    b = np.where(b.astype(np.float64) ** 2 > s, b - 1, b)
    return np.where(b < N_BINS, b, -1)


def variogram_sums(pts: np.ndarray, z: np.ndarray):
    """Per-bin sums of (z_i - z_j)^2 over pairs i < j and pair counts."""
    pts = np.asarray(pts, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    m, dim = pts.shape
    sums = np.zeros(N_BINS)
    counts = np.zeros(N_BINS, dtype=np.int64)
    for i in range(m - 1):
        d = pts[i + 1:] - pts[i]
        h2 = d[:, 0] * d[:, 0]
        for k in range(1, dim):
            h2 = h2 + d[:, k] * d[:, k]
        b = pair_bins(h2)
        dz = z[i + 1:] - z[i]
        keep = b >= 0
        np.add.at(sums, b[keep], dz[keep] * dz[keep])
        np.add.at(counts, b[keep], 1)
    return sums, counts


def variogram_features(pts: np.ndarray, z: np.ndarray, idx=None) -> np.ndarray:
    """The 33 features of one field (float64); idx: the subset of points used."""
    pts = np.asarray(pts, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    if idx is not None:
        pts, z = pts[idx], z[idx]
    sums, counts = variogram_sums(pts, z)
    f = np.zeros(N_FEAT)
    nz = counts > 0
    gamma = sums[nz] / (2.0 * counts[nz])
    f[:N_BINS][nz] = np.log(np.maximum(gamma, 1e-30))
    f[N_BINS] = np.log(float(len(z)))
    return f


# ------------------------------------------------------------- network -----
def unpack(params: np.ndarray):
    """Flat vector -> [(W, b)] per layer (views)."""
    out, off = [], 0
    for i, o in LAYERS:
        W = params[off:off + i * o].reshape(o, i)
        off += i * o
        b = params[off:off + o]
        off += o
        out.append((W, b))
    assert off == len(params)
    return out


def forward(params: np.ndarray, X: np.ndarray):
    """Activations [X, H1, H2, H3] and the output Y for standardised inputs X."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(np.asarray(params, dtype=np.float64))
    for li, (W, b) in enumerate(layers):
        a = acts[-1] @ W.T + b
        if li < len(layers) - 1:
            acts.append(np.tanh(a))
        else:
            return acts, a
    raise AssertionError


def loss(params: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    _, Y = forward(params, X)
    return float(np.mean((Y - T) ** 2))


def loss_and_grad(params: np.ndarray, X: np.ndarray, T: np.ndarray):
    """Mean squared error and its gradient with respect to the flat parameters
    (backpropagation: the chain rule through each layer in reverse)."""
    params = np.asarray(params, dtype=np.float64)
    layers = unpack(params)
    acts, Y = forward(params, X)
    B, K = Y.shape
    E = Y - np.asarray(T, dtype=np.float64)
    L = float(np.sum(E * E) / (B * K))
    dA = 2.0 * E / (B * K)                   # d loss / d (pre-activation of the output layer)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        Xin = acts[li]
        grads.append((dA.T @ Xin, dA.sum(axis=0)))
        if li > 0:
            dA = (dA @ W) * (1.0 - Xin * Xin)   # through tanh: d tanh = 1 - tanh^2
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam_step(params, grad, m, v, t: int, lr: float):
    """One Adam update (step t >= 1); returns new (params, m, v)."""
    m = BETA1 * m + (1.0 - BETA1) * grad
    v = BETA2 * v + (1.0 - BETA2) * grad * grad
    mhat = m / (1.0 - BETA1 ** t)
    vhat = v / (1.0 - BETA2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


def standardise(x, mu, sd):
    return (np.asarray(x, dtype=np.float64) - mu) / sd


def norm_stats(a: np.ndarray, flat: float = 1e-6):
    """Column means and standard deviations (population); a column whose
    deviation is below 1e-6 gets the scale `flat` (1e30 for features: a
    feature constant over the training data carries no information and is
    switched off; 1e-6 for targets)."""
    a = np.asarray(a, dtype=np.float64)
    mu = a.mean(axis=0)
    sd = np.sqrt(np.mean((a - mu) ** 2, axis=0))
    return mu, np.where(sd < 1e-6, flat, sd)
