"""Pins of two oracle helpers that the GPU tests lean on.

densify.densify_lower (rebuild a matrix from its H blocks, Section 2's block
partition): a hand-worked 3 x 3 example; the exact blocks of a covariance
matrix on the oracle's own block partition (dense blocks copied, low-rank
blocks as full-rank factorisations) give the matrix back; the lower-only form
gives the lower triangle. Planted mistakes (no mirroring, low-rank blocks not
mirrored, the upper triangle of a diagonal block) each fail a pin.

mle.fit (Nelder-Mead in the Section 5.1 coordinates, simplex x0, x0 + e_i,
box of the parameters): a quadratic objective with a known minimiser run
through the same wrapper; the first five evaluations are the initial
simplex; points outside the parameter box score +inf; on a single
observation the fit reaches the closed-form maximum of eq. (1),
-1/2 log(2 pi) - 1/2 log(z^2) - 1/2 (attained wherever sigma^2 + tau^2 = z^2).
Planted mistakes (the sign of the reported optimum, a halved simplex step, a
widened box) each fail a pin.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, densify, mle, reparam, structure


# ------------------------------------------------------------ densify ------
def _hand_blocks():
    dblocks = [(0, 0, np.array([[4.0, 9.0], [1.0, 3.0]])), (2, 2, np.array([[5.0]]))]
    lblocks = [(2, 0, np.array([[2.0]]), np.array([[1.0], [3.0]]))]
    return dblocks, lblocks


def pin_hand(fn):
    d, l = _hand_blocks()
    want = np.array([[4.0, 1.0, 2.0], [1.0, 3.0, 6.0], [2.0, 6.0, 5.0]])
    np.testing.assert_array_equal(fn(3, d, l), want)
    np.testing.assert_array_equal(fn(3, d, l, symmetric=False), np.tril(want))


def _partition_blocks():
    rng = synth.rng_for(synth.W_TESTS, 950)
    pts = synth.uniform_points(300, 2, rng)
    tree = structure.cluster_tree(pts, 16)
    bt = structure.block_tree(tree, 2.0)
    pp = pts[tree.perm]
    C = dense.covariance(pp, (1.0, 0.1, 0.5, 0.01))
    dblocks, lblocks = [], []
    for t, s in bt.dense:
        r0, r1, c0, c1 = tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s]
        D = C[r0:r1, c0:c1].copy()
        if t == s:
            D = D + 7.0 * np.triu(np.ones_like(D), 1)   # the upper part of a diagonal block is ignored
        dblocks.append((int(r0), int(c0), D))
    for t, s in bt.lowrank:
        r0, r1, c0, c1 = tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s]
        Uf, sv, Vt = np.linalg.svd(C[r0:r1, c0:c1], full_matrices=False)
        lblocks.append((int(r0), int(c0), Uf * sv, Vt.T))
    return C, dblocks, lblocks


def pin_partition(fn):
    C, d, l = _partition_blocks()
    A = fn(C.shape[0], d, l)
    assert np.abs(A - C).max() <= 1e-13 * np.abs(C).max()
    L = fn(C.shape[0], d, l, symmetric=False)
    assert np.abs(L - np.tril(C)).max() <= 1e-13 * np.abs(C).max()


DENSIFY_PINS = [pin_hand, pin_partition]


def test_densify_pins():
    for pin in DENSIFY_PINS:
        pin(densify.densify_lower)


def _mut_densify(kind):
    def fn(n, dense_blocks, lowrank_blocks, symmetric=True):
        A = np.zeros((n, n))
        for r0, c0, D in dense_blocks:
            D = np.asarray(D, dtype=np.float64)
            m, k = D.shape
            if r0 == c0:
                part = np.triu(D) if kind == "upper_diag" else np.tril(D)
                A[r0:r0 + m, c0:c0 + k] = part + (np.tril(D, -1).T if symmetric else 0.0)
            else:
                A[r0:r0 + m, c0:c0 + k] = D
                if symmetric and kind != "no_mirror":
                    A[c0:c0 + k, r0:r0 + m] = D.T
        for r0, c0, U, V in lowrank_blocks:
            B = U @ V.T
            m, k = B.shape
            A[r0:r0 + m, c0:c0 + k] = B
            if symmetric and kind not in ("no_mirror", "lowrank_unmirrored"):
                A[c0:c0 + k, r0:r0 + m] = B.T
        return A
    return fn


@pytest.mark.parametrize("kind", ["no_mirror", "lowrank_unmirrored", "upper_diag"])
def test_densify_mutations_are_caught(kind):
    failed = 0
    for pin in DENSIFY_PINS:
        try:
            pin(_mut_densify(kind))
        except AssertionError:
            failed += 1
    assert failed >= 1, kind


# ---------------------------------------------------------------- fit ------
X_STAR = np.array([-0.7, 1.3, 2.2, 9.5])
WEIGHTS = np.array([1.0, 2.0, 0.5, 0.25])


def _quadratic(x, pts, z):
    return float(np.sum(WEIGHTS * (np.asarray(x) - X_STAR) ** 2)) + 3.0


def pin_quadratic(fit_fn):
    res = fit_fn(None, None, objective=_quadratic, tol=1e-8, max_iter=2000)
    assert np.abs(res["x"] - X_STAR).max() <= 1e-3, res["x"]
    assert abs(res["logL"] - (-3.0)) <= 1e-6, res["logL"]


def pin_simplex(fit_fn):
    seen = []

    def rec(x, pts, z):
        seen.append(np.array(x, dtype=np.float64))
        return _quadratic(x, pts, z)
    fit_fn(None, None, objective=rec, max_iter=3)
    x0 = np.array(reparam.PAPER_START)
    want = [x0] + [x0 + np.eye(4)[i] for i in range(4)]
    first = seen[:5]
    for w in want:
        assert any(np.array_equal(w, s) for s in first), (w, first)


def pin_box(neg_fn):
    inside = reparam.from_theta((1.0, 0.1, 0.5, 0.01))
    pts = synth.uniform_points(5, 2, synth.rng_for(synth.W_TESTS, 951))
    z = np.ones(5)
    assert np.isfinite(neg_fn(np.array(inside), pts, z))
    for theta in [(1.0, 0.1, 8.5, 0.01), (1.0, 0.1, 0.04, 0.01), (1.0, 11.0, 0.5, 0.01), (1.0, 5e-5, 0.5, 0.01),
                  (2e6, 0.1, 0.5, 0.01), (5e-7, 0.1, 0.5, 0.01), (1.0, 0.1, 0.5, 2e3)]:
        assert neg_fn(np.array(reparam.from_theta(theta)), pts, z) == np.inf, theta


def pin_single_observation(fit_fn):
    pts = np.array([[0.3, 0.4]])
    z = np.array([1.5])
    res = fit_fn(pts, z, tol=1e-10, max_iter=2000)
    best = -0.5 * math.log(2 * math.pi) - 0.5 * math.log(z[0] ** 2) - 0.5
    assert abs(res["logL"] - best) <= 1e-6, (res["logL"], best)
    s2, _, _, t2 = res["theta"]
    assert abs(s2 + t2 - z[0] ** 2) <= 1e-3
    assert abs(dense.loglik(pts, z, res["theta"])[0] - res["logL"]) <= 1e-12


def test_fit_pins():
    pin_quadratic(mle.fit)
    pin_simplex(mle.fit)
    pin_box(mle.negloglik)
    pin_single_observation(mle.fit)


def _mut_fit(kind):
    from scipy import optimize

    def in_box(theta):
        if kind == "wide_box":
            s2, ell, nu, t2 = theta
            return 1e-9 <= s2 <= 1e9 and 1e-6 <= ell <= 100 and 0.01 <= nu <= 80 and 0 <= t2 <= 1e5
        return mle.in_box(theta)

    def neg(x, pts, z):
        theta = reparam.to_theta(x)
        if not in_box(theta):
            return np.inf
        try:
            return -dense.loglik(pts, z, theta)[0]
        except dense.NotSPD:
            return np.inf

    def fit(pts, z, x0=reparam.PAPER_START, max_iter=400, tol=1e-4, objective=None):
        f = neg if objective is None else objective
        x0 = np.asarray(x0, dtype=np.float64)
        step = 0.5 if kind == "half_step" else 1.0
        simplex = np.vstack([x0] + [x0 + step * np.eye(4)[i] for i in range(4)])
        res = optimize.minimize(f, x0, args=(pts, z), method="Nelder-Mead",
                                options={"initial_simplex": simplex, "xatol": tol, "fatol": tol,
                                         "maxiter": max_iter, "maxfev": 10 * max_iter})
        val = float(res.fun) if kind == "sign" else -float(res.fun)
        return {"x": res.x, "theta": reparam.to_theta(res.x), "logL": val}
    return fit, neg


@pytest.mark.parametrize("kind", ["sign", "half_step", "wide_box"])
def test_fit_mutations_are_caught(kind):
    fit, neg = _mut_fit(kind)
    failed = 0
    for pin, arg in [(pin_quadratic, fit), (pin_simplex, fit), (pin_box, neg), (pin_single_observation, fit)]:
        try:
            pin(arg)
        except AssertionError:
            failed += 1
    assert failed >= 1, kind
