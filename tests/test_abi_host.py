"""CPU tests of the C ABI: the library loads, exports every symbol the header
declares, and its host-side structure (cluster tree, block tree) equals the
oracle's integer-exactly. No compute call needs a GPU here."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import structure

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    import paper_2104_07146_amd as h
    return h


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "hmle.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hmle_[a-z_]+)\s*\(", src)))


def test_header_symbols_exported():
    h = _lib()
    L = h.lib()
    names = declared_symbols()
    assert "hmle_build_tree" in names and "hmle_fit" in names
    for name in names:
        getattr(L, name)          # raises AttributeError if missing
    assert set(names) == set(h.EXPORTED)


def test_default_opts():
    h = _lib()
    o = h.default_opts()
    assert (o.leaf_size, o.eta, o.aca_tol, o.max_rank, o.precision) == (64, 2.0, 1e-6, 32, 0)


@pytest.mark.parametrize("n,d,leaf,eta,gen", [(2000, 2, 64, 2.0, "unif"), (3000, 3, 32, 2.0, "unif"),
                                              (5000, 2, 128, 2.0, "clu"), (777, 2, 16, 0.8, "unif"),
                                              (129, 2, 64, 2.0, "unif"), (1, 2, 64, 2.0, "unif"),
                                              (4096, 2, 64, 2.0, "grid")])
def test_structure_matches_oracle(n, d, leaf, eta, gen):
    h = _lib()
    rng = synth.rng_for(synth.W_TESTS, 300 + n + d)
    if gen == "unif":
        pts = synth.uniform_points(n, d, rng)
    elif gen == "clu":
        pts = synth.clustered_points(n, rng)
    else:
        pts = synth.jittered_grid_points(64, 64, rng)
    s = h.Structure(pts, leaf_size=leaf, eta=eta)
    perm, nodes, bmin, bmax = s.export_tree()
    tree = structure.cluster_tree(pts, leaf)
    np.testing.assert_array_equal(perm, tree.perm)
    np.testing.assert_array_equal(nodes[:, 0], tree.lo)
    np.testing.assert_array_equal(nodes[:, 1], tree.hi)
    np.testing.assert_array_equal(nodes[:, 2:], tree.child)
    np.testing.assert_array_equal(bmin, tree.bmin)
    np.testing.assert_array_equal(bmax, tree.bmax)
    dense, lowrank = s.export_blocks()
    bt = structure.block_tree(tree, eta)
    np.testing.assert_array_equal(dense, bt.dense)
    np.testing.assert_array_equal(lowrank, bt.lowrank)


def test_structure_rejects_bad_input():
    h = _lib()
    pts = np.zeros((10, 2))
    with pytest.raises(h.HmleError):
        h.Structure(pts, leaf_size=0)
    with pytest.raises(h.HmleError):
        h.Structure(np.zeros((10, 4)))
    bad = pts.copy()
    bad[3, 1] = np.nan
    with pytest.raises(h.HmleError):
        h.Structure(bad)


def test_plan_stats_consistent():
    h = _lib()
    pts = synth.uniform_points(2000, 2, synth.rng_for(synth.W_SMALL_UNIFORM))
    s = h.Structure(pts, leaf_size=64, eta=2.0)
    st = s.plan_stats()
    tree = structure.cluster_tree(pts, 64)
    bt = structure.block_tree(tree, 2.0)
    dense_entries = sum(int(tree.hi[t] - tree.lo[t]) * int(tree.hi[u] - tree.lo[u]) for t, u in bt.dense)
    lr_dims = sum(int(tree.hi[t] - tree.lo[t]) + int(tree.hi[u] - tree.lo[u]) for t, u in bt.lowrank)
    assert st["dense_entries"] == dense_entries
    assert st["lr_dims"] == lr_dims
    assert st["leaves"] == 32
    assert st["pairs"] > 0 and st["lr_pairs"] <= st["pairs"]
