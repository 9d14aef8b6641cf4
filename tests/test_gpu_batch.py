"""GPU tests of batched evaluation (many independent problems in one plan).

Each problem of a batch must give exactly what it gives alone (same trees,
blocks, test matrices and summation order): compared bit for bit, through the
staged calls and through the graph-replayed hmle_eval_batch, over two
replays with different parameters. Against the dense float64 oracle the
single-problem tolerance applies. A problem that is not positive definite is
reported on its own without disturbing the others.
"""
import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu


def _h():
    import paper_2104_07146_amd as h
    h.lib()
    return h


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


SIZES = [500, 1337, 64, 2900, 5, 800, 1]


def _problems(seed, sizes=SIZES):
    rng = synth.rng_for(synth.W_BATCH, seed)
    pts_list, thetas, zs = [], [], []
    for n in sizes:
        pts = synth.uniform_points(n, 2, rng)
        th = synth.batch_theta(rng)
        w = synth.standard_normal(n, rng)
        pts_list.append(pts)
        thetas.append(th)
        zs.append(dense.sample(pts, th, w))
    return pts_list, thetas, zs


def _singles(h, pts_list, thetas, zs, **opts):
    res = []
    for pts, th, z in zip(pts_list, thetas, zs):
        with h.Problem(_cuda(pts), **opts) as p:
            res.append(p.eval(th, _cuda(z)))
    return np.array(res)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_problems(precision):
    h = _h()
    prec = h.FP64 if precision == "fp64" else h.MIXED
    opts = dict(leaf_size=64, eta=2.0, aca_tol=1e-6, max_rank=32, precision=prec)
    pts_list, thetas, zs = _problems(1)
    print(f"batch sizes={SIZES} precision={precision}", flush=True)
    single = _singles(h, pts_list, thetas, zs, **opts)
    z = _cuda(np.concatenate(zs))
    with h.Batch([_cuda(p) for p in pts_list], **opts) as b:
        assert b.plan_stats()["steps"] == max(h.Structure(p, leaf_size=64).plan_stats()["leaves"] for p in pts_list)
        # staged calls
        b.assemble(thetas)
        st = b.factor()
        assert (st == h.HMLE_OK).all()
        out, st = b.loglik(z)
        assert (st == h.HMLE_OK).all()
        np.testing.assert_array_equal(out, single)
        # graph capture, then replays with other parameters
        out, st = b.eval(thetas, z)
        np.testing.assert_array_equal(out, single)
        thetas2 = [(s2 * 1.1, ell * 0.9, nu, t2 * 1.3) for s2, ell, nu, t2 in thetas]
        single2 = _singles(h, pts_list, thetas2, zs, **opts)
        for rep in range(3):
            out2, st2 = b.eval(thetas2 if rep % 2 == 0 else thetas, z)
            np.testing.assert_array_equal(out2, single2 if rep % 2 == 0 else single)
    if precision == "fp64":
        for q, (pts, th, zq) in enumerate(zip(pts_list, thetas, zs)):
            ref = dense.loglik(pts, zq, th)
            assert abs(single[q, 0] - ref[0]) <= 2e-5 * abs(ref[0]), (q, single[q, 0], ref[0])


def test_batch_not_spd_is_per_problem():
    h = _h()
    pts_list, thetas, zs = _problems(2, sizes=[300, 4, 700])
    # problem 1: a repeated point and no nugget -> singular matrix
    pts_list[1] = np.array([[0.2, 0.2], [0.2, 0.2], [0.7, 0.1], [0.4, 0.9]])
    thetas[1] = (1.0, 0.3, 0.5, 0.0)
    zs[1] = np.ones(4)
    opts = dict(leaf_size=64, aca_tol=1e-6)
    z = _cuda(np.concatenate(zs))
    with h.Batch([_cuda(p) for p in pts_list], **opts) as b:
        out, st = b.eval(thetas, z)
        assert list(st) == [h.HMLE_OK, h.HMLE_E_NOT_SPD, h.HMLE_OK]
        assert np.isnan(out[1]).all()
        keep = [0, 2]
        single = _singles(h, [pts_list[q] for q in keep], [thetas[q] for q in keep], [zs[q] for q in keep], **opts)
        np.testing.assert_array_equal(out[keep], single)
        # the same batch recovers with a nugget
        thetas[1] = (1.0, 0.3, 0.5, 0.1)
        out, st = b.eval(thetas, z)
        assert (st == h.HMLE_OK).all()
        ref = dense.loglik(pts_list[1], zs[1], thetas[1])
        assert abs(out[1, 0] - ref[0]) <= 1e-12 * abs(ref[0])


def test_batch_sampler_equals_single():
    h = _h()
    import torch
    pts_list, thetas, _ = _problems(3, sizes=[900, 130, 2000])
    rng = synth.rng_for(synth.W_BATCH, 33)
    ws = [synth.standard_normal(len(p), rng) for p in pts_list]
    opts = dict(leaf_size=64, aca_tol=1e-8, max_rank=48)
    with h.Batch([_cuda(p) for p in pts_list], **opts) as b:
        b.assemble(thetas)
        assert (b.factor() == h.HMLE_OK).all()
        zb = b.sample(_cuda(np.concatenate(ws))).cpu().numpy()
    for q, (pts, th, w) in enumerate(zip(pts_list, thetas, ws)):
        with h.Problem(_cuda(pts), **opts) as p:
            p.assemble(th)
            p.factor()
            zs = p.sample(_cuda(w)).cpu().numpy()
        np.testing.assert_array_equal(zb[b.offsets[q]:b.offsets[q + 1]], zs)


def test_batch_validation():
    h = _h()
    pts_list, thetas, zs = _problems(4, sizes=[100, 200])
    with h.Batch([_cuda(p) for p in pts_list], leaf_size=64) as b:
        bad = list(thetas)
        bad[1] = (1.0, -0.1, 0.5, 0.01)
        with pytest.raises(h.HmleError) as e:
            b.eval(bad, _cuda(np.concatenate(zs)))
        assert "problem 1" in str(e.value)
        with pytest.raises(ValueError):
            b.assemble(thetas[:1])
        import ctypes
        out = (ctypes.c_double * 3)()
        zc = _cuda(np.concatenate(zs))
        assert h.lib().hmle_loglik(b._h, zc.data_ptr(), out) == h.HMLE_E_INVALID


def test_batch_512_problems_sampled():
    """The batched workload at full size: 512 problems, n ~ U{500..8000},
    own points and parameters (leaf 64, eta 2, eps 1e-6). Data: each problem's
    field drawn by the batch's own sampler at eps 1e-8 (the dense draws would
    take the host minutes). Sampled problems are compared bit for bit with the
    same problem alone, and the smallest with the dense oracle."""
    h = _h()
    import torch
    specs = synth.batch_problem_specs(512)
    pts_list, thetas = [], []
    for sp in specs:
        rng = synth.rng_for(synth.W_BATCH, 1000 + sp["seed_sub"])
        pts_list.append(synth.uniform_points(sp["n"], 2, rng))
        thetas.append(sp["theta"])
    total = sum(len(p) for p in pts_list)
    print(f"512 problems, {total} points", flush=True)
    w = synth.standard_normal(total, synth.rng_for(synth.W_BATCH, 999))
    with h.Batch([_cuda(p) for p in pts_list], leaf_size=64, aca_tol=1e-8, max_rank=48) as bs:
        bs.assemble(thetas)
        assert (bs.factor() == h.HMLE_OK).all()
        z = bs.sample(_cuda(w))
    opts = dict(leaf_size=64, eta=2.0, aca_tol=1e-6, max_rank=32)
    with h.Batch([_cuda(p) for p in pts_list], **opts) as b:
        out, st = b.eval(thetas, z)
        assert (st == h.HMLE_OK).all()
        assert np.isfinite(out).all()
        out2, _ = b.eval(thetas, z)
        np.testing.assert_array_equal(out, out2)
        zs = [t.cpu().numpy() for t in b.split(z)]
    pick = [0, 137, 511, int(np.argmin([len(p) for p in pts_list]))]
    for q in pick:
        with h.Problem(_cuda(pts_list[q]), **opts) as p:
            one = p.eval(thetas[q], _cuda(zs[q]))
        np.testing.assert_array_equal(out[q], np.array(one))
    q = pick[-1]
    ref = dense.loglik(pts_list[q], zs[q], thetas[q])
    assert abs(out[q, 0] - ref[0]) <= 2e-5 * abs(ref[0]), (q, out[q, 0], ref[0])
