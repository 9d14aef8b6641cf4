"""The seeded input generators (synth/), which both the oracle-side tests and
the GPU path draw from: the recipe stated for each workload holds, and every
stream is reproducible."""
import math

import numpy as np
import pytest

import synth


def test_streams_are_reproducible_and_distinct():
    a = synth.rng_for(synth.W_TESTS, 7).random(5)
    b = synth.rng_for(synth.W_TESTS, 7).random(5)
    c = synth.rng_for(synth.W_TESTS, 8).random(5)
    d = synth.rng_for(synth.W_CLUSTERED, 7).random(5)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)


def test_uniform_points():
    p = synth.uniform_points(1000, 3, synth.rng_for(synth.W_TESTS, 1))
    assert p.shape == (1000, 3) and p.dtype == np.float64 and p.flags.c_contiguous
    assert p.min() >= 0.0 and p.max() < 1.0


def test_jittered_grid_cells():
    nx, ny = 37, 23
    p = synth.jittered_grid_points(nx, ny, synth.rng_for(synth.W_JITTERED_GRID, 1))
    assert p.shape == (nx * ny, 2) and p.flags.c_contiguous
    k = np.arange(nx * ny)
    cx, cy = (k % nx + 0.5) / nx, (k // nx + 0.5) / ny       # row-major over (iy, ix)
    assert np.all(np.abs(p[:, 0] - cx) <= 0.4 / nx + 1e-15)
    assert np.all(np.abs(p[:, 1] - cy) <= 0.4 / ny + 1e-15)
    # the jitter fills its range: some point moved by more than 0.35 cells on each axis
    assert np.max(np.abs(p[:, 0] - cx)) * nx > 0.35 and np.max(np.abs(p[:, 1] - cy)) * ny > 0.35


def test_the_256k_grid():
    p = synth.jittered_grid_points(512, 500, synth.rng_for(synth.W_JITTERED_GRID))
    assert p.shape == (256_000, 2)
    assert p.min() > 0.0 and p.max() < 1.0
    # points of neighbouring cells stay 0.2 cell widths apart (jitter 0.4 each
    # way); checked on neighbours in (y, x) order
    q = p[np.lexsort((p[:, 0], p[:, 1]))]
    assert np.min(np.linalg.norm(np.diff(q, axis=0), axis=1)) > 0.2 / 512


def test_clustered_points_inhomogeneous():
    n = 64_000
    p = synth.clustered_points(n, synth.rng_for(synth.W_CLUSTERED))
    assert p.shape == (n, 2) and p.min() >= 0.0 and p.max() <= 1.0
    counts = np.histogram2d(p[:, 0], p[:, 1], bins=20, range=[[0, 1], [0, 1]])[0].ravel()
    # 30 % uniform: every cell holds at least its uniform share, minus sampling noise
    assert counts.min() >= 0.3 * n / 400 * 0.6
    # 70 % in eight tight clusters: the occupancy is far from uniform (a uniform
    # draw has a coefficient of variation of about 0.08 here)
    assert counts.std() / counts.mean() > 1.0


def test_collinear_points():
    p, t, u = synth.collinear_points(500, 3, synth.rng_for(synth.W_TESTS, 2), length=2.0)
    assert abs(np.linalg.norm(u) - 1.0) < 1e-15
    assert np.all(np.diff(t) >= 0) and t.min() >= 0 and t.max() <= 2.0
    np.testing.assert_array_equal(p, t[:, None] * u[None, :])
    assert np.linalg.matrix_rank(p, tol=1e-12) == 1


def test_batch_specs():
    specs = synth.batch_problem_specs(512)
    assert specs == synth.batch_problem_specs(512)
    sizes = np.array([s["n"] for s in specs])
    assert sizes.min() >= 500 and sizes.max() <= 8000
    assert 2.0e6 < sizes.sum() < 2.3e6
    assert [s["seed_sub"] for s in specs] == list(range(1, 513))
    th = np.array([s["theta"] for s in specs])
    lo, hi = np.array([0.5, 0.05, 0.3, 1e-3]), np.array([2.0, 0.3, 2.0, 0.1])
    assert np.all(th >= lo) and np.all(th <= hi)


def test_subsets_init_and_order():
    rng = synth.rng_for(synth.W_TESTS, 3)
    idx = synth.subset_indices(10_000, 4096, rng)
    assert idx.dtype == np.int32 and len(np.unique(idx)) == 4096 and np.all(np.diff(idx) > 0)
    assert np.array_equal(synth.subset_indices(100, 4096, rng), np.arange(100))
    w = synth.mlp_init(rng)
    assert w.dtype == np.float32 and w.size == 33 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 4 + 4 == 37892
    assert np.all(w[33 * 128: 33 * 128 + 128] == 0) and np.abs(w[:33 * 128]).max() <= np.sqrt(6 / 161)
    perm = synth.minibatch_order(1000, rng)
    assert perm.dtype == np.int32 and np.array_equal(np.sort(perm), np.arange(1000))


def test_g_and_h_closed_forms():
    z = np.linspace(-4, 4, 801)
    # g = h = 0 is the Gaussian field itself, shifted and scaled
    np.testing.assert_array_equal(synth.tukey_g_and_h(z, 1.0, 2.0, 0.0, 0.0), 1.0 + 2.0 * z)
    # continuity at g = 0 and the mirror symmetry T_{-g}(-z) - xi = -(T_g(z) - xi)
    t0 = synth.tukey_g_and_h(z, 0.0, 1.0, 0.0, 0.2)
    np.testing.assert_allclose(synth.tukey_g_and_h(z, 0.0, 1.0, 1e-7, 0.2), t0, rtol=0, atol=1e-5)
    for _, _, g, h in synth.G_AND_H_TEST2A:
        tp = synth.tukey_g_and_h(z, 1.0, 2.0, g, h) - 1.0
        tm = synth.tukey_g_and_h(-z, 1.0, 2.0, -g, h) - 1.0
        np.testing.assert_allclose(tm, -tp, rtol=1e-14, atol=1e-14)
        assert np.all(np.diff(tp) > 0)           # strictly increasing for h >= 0
        assert synth.tukey_g_and_h(np.array([0.0]), 1.0, 2.0, g, h)[0] == 1.0   # the median maps to xi


@pytest.mark.parametrize("xi,omega,g,h", [(0.0, 1.0, 0.5, 0.0), (1.0, 2.0, 0.0, 0.1), (1.0, 2.0, 0.0, 0.2)])
def test_g_and_h_moments(xi, omega, g, h):
    """Monte Carlo against closed forms for Z ~ N(0, 1): with h = 0,
    E T = xi + omega (e^{g^2/2} - 1) / g; with g = 0, E T = xi and
    Var T = omega^2 (1 - 2h)^{-3/2} (h < 1/2; the check of the sample variance
    needs a finite fourth moment, h < 1/4)."""
    n = 2_000_000
    z = synth.rng_for(synth.W_TESTS, 990).standard_normal(n)
    t = synth.tukey_g_and_h(z, xi, omega, g, h)
    se = t.std() / math.sqrt(n)
    if h == 0.0:
        assert abs(t.mean() - (xi + omega * (math.exp(g * g / 2) - 1) / g)) <= 5 * se
    else:
        assert abs(t.mean() - xi) <= 5 * se
        var = omega ** 2 * (1 - 2 * h) ** -1.5
        # standard error of the sample variance from the fourth moment, E[Z^4 e^{2hZ^2}] = 3 (1 - 4h)^{-5/2}
        m4 = omega ** 4 * 3 * (1 - 4 * h) ** -2.5
        assert abs(t.var() - var) <= 5 * math.sqrt((m4 - var * var) / n)


def test_g_and_h_test2a_parameters():
    assert synth.G_AND_H_TEST2A == ((1.0, 2.0, 0.2, 0.2), (1.0, 2.0, 0.5, 0.3))

