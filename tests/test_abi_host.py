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
    assert (o.pair_chunk, o.sketch_group, o.spd_margin) == (1, 8, -1.0)   # -1: automatic floor


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


def test_batch_structure_is_the_union_of_single_structures():
    """A batch's merged trees are each problem's own trees shifted by the node
    and point offsets; plan counts add up; the batch takes as many steps as its
    largest problem has leaves."""
    h = _lib()
    rng = synth.rng_for(synth.W_BATCH, 11)
    sizes = [700, 65, 1, 2100, 1300]
    pts_list = [synth.uniform_points(n, 2, rng) for n in sizes]
    b = h.BatchStructure(pts_list, leaf_size=64, eta=2.0)
    perm, nodes, bmin, bmax = b.export_tree()
    dense, lowrank = b.export_blocks()
    node0 = pt0 = 0
    d0 = l0 = 0
    tot = {k: 0 for k in ["pairs", "inner", "dense_entries", "lr_dims", "leaves", "grams", "col_solves"]}
    max_leaves = 0
    for pts in pts_list:
        s = h.Structure(pts, leaf_size=64, eta=2.0)
        sp, sn, smin, smax = s.export_tree()
        sd, sl = s.export_blocks()
        k = len(sn)
        np.testing.assert_array_equal(perm[pt0:pt0 + len(pts)], sp + pt0)
        np.testing.assert_array_equal(nodes[node0:node0 + k, :2], sn[:, :2] + pt0)
        ch = sn[:, 2:].copy()
        ch[ch >= 0] += node0
        np.testing.assert_array_equal(nodes[node0:node0 + k, 2:], ch)
        np.testing.assert_array_equal(bmin[node0:node0 + k], smin)
        np.testing.assert_array_equal(bmax[node0:node0 + k], smax)
        np.testing.assert_array_equal(dense[d0:d0 + len(sd)], sd + node0)
        np.testing.assert_array_equal(lowrank[l0:l0 + len(sl)], sl + node0)
        st = s.plan_stats()
        for key in tot:
            tot[key] += st[key]
        max_leaves = max(max_leaves, st["leaves"])
        assert st["steps"] == st["leaves"] and st["problems"] == 1
        node0 += k
        pt0 += len(pts)
        d0 += len(sd)
        l0 += len(sl)
    bs = b.plan_stats()
    for key in tot:
        assert bs[key] == tot[key], key
    assert bs["steps"] == max_leaves and bs["problems"] == len(sizes)


def test_batch_rejects_bad_offsets():
    h = _lib()
    with pytest.raises(h.HmleError):
        h.BatchStructure([np.zeros((3, 2)), np.zeros((0, 2))])


def test_default_fit_opts():
    import ctypes
    h = _lib()
    o = h.FitOpts()
    h.lib().hmle_default_fit_opts(ctypes.byref(o))
    assert (o.max_iter, o.tol, o.step, o.use_backoff, o.report_every, o.profile_variance) == (400, 1e-4, 1.0, 1, 0, 0)


def test_fit_batch_and_predict_validate_without_gpu():
    """Argument and state errors come back as status codes before any device work."""
    import ctypes
    h = _lib()
    L = h.lib()
    assert L.hmle_fit_batch(None, None, None, None, None, None, None) == h.HMLE_E_INVALID
    assert L.hmle_predict(None, None, None, 0, None) == h.HMLE_E_INVALID
    pts = synth.uniform_points(100, 2, synth.rng_for(synth.W_TESTS, 950))
    with h.Structure(pts, leaf_size=16) as s:
        z = np.zeros(100)
        th = h.Theta()
        assert L.hmle_predict(s._h, z.ctypes.data, None, -1, None) == h.HMLE_E_INVALID
        assert L.hmle_predict(s._h, z.ctypes.data, z.ctypes.data, 1, z.ctypes.data) == h.HMLE_E_STATE
        assert L.hmle_fit_batch(s._h, z.ctypes.data, None, None, ctypes.byref(th), None, None) == h.HMLE_E_STATE


def test_fit_resumable_validates_without_gpu():
    """The checkpointed fit refuses a missing or wrongly sized buffer and a
    checkpoint of another problem size before any work; with a fresh buffer it
    reaches the first evaluation, which a structure-only problem refuses
    (E_STATE), and the buffer stays as it was."""
    import ctypes
    import struct
    h = _lib()
    L = h.lib()
    pts = synth.uniform_points(100, 2, synth.rng_for(synth.W_TESTS, 951))
    with h.Structure(pts, leaf_size=16) as s:
        z = np.zeros(100)
        th = h.Theta()
        buf = ctypes.create_string_buffer(h.FIT_STATE_BYTES)
        assert L.hmle_fit_resumable(s._h, z.ctypes.data, None, None, None, h.FIT_STATE_BYTES,
                                    ctypes.byref(th), None) == h.HMLE_E_INVALID
        assert L.hmle_fit_resumable(s._h, z.ctypes.data, None, None, buf, h.FIT_STATE_BYTES - 8,
                                    ctypes.byref(th), None) == h.HMLE_E_INVALID
        assert L.hmle_fit_resumable(s._h, z.ctypes.data, None, None, buf, h.FIT_STATE_BYTES,
                                    ctypes.byref(th), None) == h.HMLE_E_STATE
        assert buf.raw == bytes(h.FIT_STATE_BYTES)
        # a checkpoint (tag, dims 4, full search) of a problem with 99 points
        other = bytearray(h.FIT_STATE_BYTES)
        other[0:8] = b"HMLEFIT1"
        struct.pack_into("<6i2d", other, 8, 4, 0, 3, 10, 0, 0, 99.0, 0.0)
        ctypes.memmove(buf, bytes(other), h.FIT_STATE_BYTES)
        assert L.hmle_fit_resumable(s._h, z.ctypes.data, None, None, buf, h.FIT_STATE_BYTES,
                                    ctypes.byref(th), None) == h.HMLE_E_INVALID
        assert buf.raw == bytes(other)
