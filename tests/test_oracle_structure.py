"""Pins of the oracle's cluster tree and block tree (Section 2's recursive
partition): invariants every valid partition satisfies, and a hand-computed
example. The GPU library's trees are compared with these integer-exactly."""
import numpy as np
import pytest

import synth
from oracle import structure


def _pts(n, d, k):
    return synth.uniform_points(n, d, synth.rng_for(synth.W_TESTS, 200 + k))


def check_tree_invariants(pts, tree, leaf):
    n = pts.shape[0]
    assert sorted(tree.perm.tolist()) == list(range(n))
    assert tree.lo[0] == 0 and tree.hi[0] == n
    for t in range(tree.n_nodes):
        p = pts[tree.perm[tree.lo[t]:tree.hi[t]]]
        np.testing.assert_array_equal(tree.bmin[t], p.min(axis=0))
        np.testing.assert_array_equal(tree.bmax[t], p.max(axis=0))
        if tree.is_leaf(t):
            assert tree.hi[t] - tree.lo[t] <= leaf
        else:
            c1, c2 = tree.child[t]
            m = tree.hi[t] - tree.lo[t]
            assert m > leaf
            assert tree.lo[c1] == tree.lo[t] and tree.hi[c1] == tree.lo[c2] and tree.hi[c2] == tree.hi[t]
            assert tree.hi[c1] - tree.lo[c1] == m // 2
            assert tree.level[c1] == tree.level[t] + 1
            # split along the longest side: the children are separated along it
            ext = tree.bmax[t] - tree.bmin[t]
            ax = int(np.argmax(ext))
            assert tree.bmax[c1, ax] <= tree.bmin[c2, ax]


def check_block_cover(tree, bt, eta):
    n = int(tree.hi[0])
    cover = np.zeros((n, n), dtype=np.int32)
    for arr, lr in ((bt.dense, False), (bt.lowrank, True)):
        for t, s in arr:
            a0, a1, b0, b1 = tree.lo[t], tree.hi[t], tree.lo[s], tree.hi[s]
            assert a0 >= b0                         # lower triangle
            cover[a0:a1, b0:b1] += 1
            if lr:
                assert t != s and structure.admissible(tree, t, s, eta)
            elif t != s:
                assert not structure.admissible(tree, t, s, eta)
                assert tree.is_leaf(t) or tree.is_leaf(s)
    low = np.tril(np.ones((n, n), dtype=np.int32))
    # diagonal blocks cover their whole square; everything in the lower triangle exactly once
    assert np.all(cover[low == 1] == 1)
    assert structure.covered_entries(tree, bt) == n * n


@pytest.mark.parametrize("n,d,leaf,eta", [(500, 2, 16, 2.0), (700, 3, 32, 2.0), (300, 2, 8, 0.7),
                                          (129, 2, 64, 2.0), (64, 2, 64, 2.0), (1, 2, 4, 2.0)])
def test_tree_and_blocks(n, d, leaf, eta):
    pts = _pts(n, d, n + d)
    tree = structure.cluster_tree(pts, leaf)
    check_tree_invariants(pts, tree, leaf)
    bt = structure.block_tree(tree, eta)
    check_block_cover(tree, bt, eta)


def test_hand_example():
    # Four points on a line, leaf size 1: root {0,1,2,3} -> {0,1},{2,3} -> singletons.
    pts = np.array([[3.0, 0.0], [0.0, 0.0], [2.0, 0.0], [1.0, 0.0]])
    tree = structure.cluster_tree(pts, 1)
    assert tree.perm.tolist() == [1, 3, 2, 0]
    assert tree.lo.tolist() == [0, 0, 2, 0, 1, 2, 3]
    assert tree.child.tolist() == [[1, 2], [3, 4], [5, 6], [-1, -1], [-1, -1], [-1, -1], [-1, -1]]
    # eta = 1: diam({0,1}) = 1 = dist({2,3},{0,1}) -> (2,1) admissible.
    bt = structure.block_tree(tree, 1.0)
    assert sorted(map(tuple, bt.dense.tolist())) == [(3, 3), (4, 4), (5, 5), (6, 6)]
    assert sorted(map(tuple, bt.lowrank.tolist())) == [(2, 1), (4, 3), (6, 5)]
    # eta = 0.5: (2,1) is refined into its four singleton pairs, all admissible.
    bt = structure.block_tree(tree, 0.5)
    assert sorted(map(tuple, bt.lowrank.tolist())) == [(4, 3), (5, 3), (5, 4), (6, 3), (6, 4), (6, 5)]


def test_tie_break_lowest_axis_and_index():
    # Equal extents on both axes -> split along axis 0; equal coordinates -> by original index.
    pts = np.array([[0.0, 0.0], [1.0, 1.0], [0.0, 1.0], [1.0, 0.0], [0.5, 0.5]])
    tree = structure.cluster_tree(pts, 2)
    # axis 0 order: x=0 -> indices 0,2 ; x=0.5 -> 4 ; x=1 -> 1,3 ; first half = 2 points
    assert tree.perm[:2].tolist() == [0, 2]
    assert sorted(tree.perm[2:].tolist()) == [1, 3, 4]


def test_sizes_of_the_2000_point_case():
    # n=2000 uniform, leaf 64: depth 5, 63 nodes, 32 leaves of 62-63 points.
    pts = synth.uniform_points(2000, 2, synth.rng_for(synth.W_SMALL_UNIFORM))
    tree = structure.cluster_tree(pts, 64)
    assert tree.n_nodes == 63 and int(tree.level.max()) == 5
    sizes = (tree.hi - tree.lo)[tree.child[:, 0] < 0]
    assert len(sizes) == 32 and sizes.min() == 62 and sizes.max() == 63
