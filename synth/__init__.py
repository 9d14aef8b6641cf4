"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module holds no arithmetic of the method: it only draws locations,
standard-normal vectors and parameter vectors. Every covariance evaluation,
factorisation or likelihood lives either in ``oracle/`` (test
infrastructure) or in the HIP library.

The paper's workloads (Section 5: unit square, 90k-900k irregular locations,
Matern parameters in the ranges of Tables 1-3) come from a competition whose
data is not available here; these generators stand in for them with the same
geometry and sizes.

RNG: NumPy PCG64 seeded from ``SeedSequence(BASE_SEED).spawn(...)``; the
child index identifies the workload so every consumer draws the same bytes.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 2104071460

# Workload identifiers (child index of the base seed sequence).
W_SMALL_UNIFORM = 1      # n=2000 uniform in the unit square
W_CLUSTERED = 2          # 8-cluster mixture + 30% uniform
W_JITTERED_GRID = 3      # jittered 2-D grid / 3-D uniform cube
W_BATCH = 4              # 512 independent small problems
W_LEARNED = 5            # learned-start training fields
W_TESTS = 9              # assorted test inputs


def rng_for(workload: int, sub: int = 0) -> np.random.Generator:
    """Generator for (workload, sub-stream); deterministic across machines."""
    ss = np.random.SeedSequence(BASE_SEED).spawn(workload + 1)[workload]
    if sub:
        ss = ss.spawn(sub + 1)[sub]
    return np.random.Generator(np.random.PCG64(ss))


def uniform_points(n: int, dim: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in [0,1]^dim, float64 row-major (n, dim)."""
    return np.ascontiguousarray(rng.random((n, dim)), dtype=np.float64)


def clustered_points(n: int, rng: np.random.Generator, n_clusters: int = 8,
                     spread: float = 0.05, uniform_frac: float = 0.3) -> np.ndarray:
    """Inhomogeneous 2-D points: (1-uniform_frac) from isotropic Gaussian
    clusters (centres uniform in [0.15,0.85]^2, std ``spread``, equal weights,
    draws outside the unit square redrawn) plus uniform_frac uniform points."""
    n_unif = int(round(uniform_frac * n))
    n_clu = n - n_unif
    centres = 0.15 + 0.7 * rng.random((n_clusters, 2))
    labels = rng.integers(0, n_clusters, size=n_clu)
    pts = np.empty((n_clu, 2))
    todo = np.arange(n_clu)
    while todo.size:
        cand = centres[labels[todo]] + spread * rng.standard_normal((todo.size, 2))
        ok = np.all((cand >= 0.0) & (cand <= 1.0), axis=1)
        pts[todo[ok]] = cand[ok]
        todo = todo[~ok]
    unif = rng.random((n_unif, 2))
    out = np.concatenate([pts, unif], axis=0)
    out = out[rng.permutation(n)]
    return np.ascontiguousarray(out, dtype=np.float64)


def jittered_grid_points(nx: int, ny: int, rng: np.random.Generator,
                         jitter: float = 0.4) -> np.ndarray:
    """Cell centres of an nx-by-ny grid on the unit square, each moved by
    U(-jitter, jitter) cell widths per axis; row-major over (iy, ix)."""
    hx, hy = 1.0 / nx, 1.0 / ny
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    cx = (ix.ravel() + 0.5) * hx
    cy = (iy.ravel() + 0.5) * hy
    jx = rng.uniform(-jitter, jitter, cx.size) * hx
    jy = rng.uniform(-jitter, jitter, cy.size) * hy
    return np.ascontiguousarray(np.stack([cx + jx, cy + jy], axis=1), dtype=np.float64)


def collinear_points(n: int, dim: int, rng: np.random.Generator,
                     length: float = 1.0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """n points on a segment s_i = t_i * u, u a random unit vector in R^dim,
    t_i sorted uniform draws on [0, length] (distinct with probability 1).
    Returns (points (n, dim), t (n,), u (dim,))."""
    u = rng.standard_normal(dim)
    u /= np.linalg.norm(u)
    t = np.sort(rng.random(n) * length)
    pts = np.ascontiguousarray(t[:, None] * u[None, :], dtype=np.float64)
    return pts, t, u


def standard_normal(n: int, rng: np.random.Generator) -> np.ndarray:
    return np.ascontiguousarray(rng.standard_normal(n), dtype=np.float64)


def batch_problem_specs(count: int = 512, seed_workload: int = W_BATCH):
    """Sizes and parameters of the batched workload: n_i ~ U{500..8000},
    sigma2 ~ U[0.5,2], range ~ U[0.05,0.3], nu ~ U[0.3,2], tau2 ~ U[1e-3,0.1].
    Returns a list of dicts with 'n', 'theta' (sigma2, range, nu, tau2) and
    'seed_sub' (the sub-stream holding that problem's points and normals)."""
    rng = rng_for(seed_workload)
    specs = []
    for i in range(count):
        n = int(rng.integers(500, 8001))
        specs.append({"n": n, "theta": batch_theta(rng), "seed_sub": i + 1})
    return specs


def batch_theta(rng: np.random.Generator):
    """One parameter draw of the batched / learned-start workloads:
    (sigma2, range, nu, tau2) ~ U[0.5,2] x U[0.05,0.3] x U[0.3,2] x U[1e-3,0.1]."""
    return (float(rng.uniform(0.5, 2.0)), float(rng.uniform(0.05, 0.3)),
            float(rng.uniform(0.3, 2.0)), float(rng.uniform(1e-3, 0.1)))


def subset_indices(n: int, m: int, rng: np.random.Generator) -> np.ndarray:
    """Sorted indices of a uniform subset of m of n points (all when n <= m):
    the points a variogram feature vector is computed from."""
    if n <= m:
        return np.arange(n, dtype=np.int32)
    return np.sort(rng.choice(n, m, replace=False)).astype(np.int32)


def mlp_init(rng: np.random.Generator, layers=((33, 128), (128, 128), (128, 128), (128, 4))) -> np.ndarray:
    """Initial weights of the start-proposal network, float32, flat in the
    order W1, b1, ..., W4, b4 (W: out x in, row-major): Glorot-uniform
    weights U[-a, a], a = sqrt(6 / (in + out)), zero biases."""
    parts = []
    for i, o in layers:
        a = np.sqrt(6.0 / (i + o))
        parts.append(rng.uniform(-a, a, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def minibatch_order(n: int, rng: np.random.Generator) -> np.ndarray:
    """A random permutation of 0..n-1 (int32): the row order of one epoch."""
    return rng.permutation(n).astype(np.int32)


# The two non-Gaussian datasets of Section 5's Test 2a (its parameter table):
# a Gaussian field with (sigma2, range, nu, tau2) = (1, 0.1, 1, 0) transformed
# by Tukey g-and-h with (xi, omega, g, h) as below.
G_AND_H_TEST2A = ((1.0, 2.0, 0.2, 0.2), (1.0, 2.0, 0.5, 0.3))


def tukey_g_and_h(z, xi: float, omega: float, g: float, h: float) -> np.ndarray:
    """Tukey g-and-h marginal transform of a standard Gaussian field z
    (Section 5, Test 2a): xi + omega * (exp(g z) - 1) / g * exp(h z^2 / 2),
    with (exp(g z) - 1) / g read as its limit z at g = 0; g sets the skewness,
    h >= 0 the tail weight."""
    z = np.asarray(z, dtype=np.float64)
    core = z if g == 0.0 else np.expm1(g * z) / g
    return np.ascontiguousarray(xi + omega * core * np.exp(0.5 * h * z * z), dtype=np.float64)

