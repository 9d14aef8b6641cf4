"""Caller-supplied device memory (hmle_build_tree_alloc / hmle_build_batch_alloc)
through the C ABI: with PyTorch's caching allocator bound as the problem's
allocator the results equal those of the library's own allocation bit for
bit, PyTorch accounts for the memory while the problem lives and gets it back
when it is destroyed (including the workspaces that later calls add); an
allocator that fails after k blocks makes the build return HMLE_E_NOMEM with
every block obtained before freed again; an allocator missing a callback is
refused."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import dense

pytestmark = pytest.mark.gpu


def _cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_torch_allocator_same_results_and_accounting():
    import torch
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 740)
    pts = synth.uniform_points(3000, 2, rng)
    theta = (1.0, 0.1, 0.8, 0.02)
    z = dense.sample(pts, theta, synth.standard_normal(3000, rng))
    dp, dz = _cuda(pts), _cuda(z)
    new = _cuda(synth.uniform_points(50, 2, rng))
    print("allocator: default", flush=True)
    with h.Problem(dp, leaf_size=64, aca_tol=1e-7) as p:
        ref = p.eval(theta, dz)
        ref_pred = p.predict(dz, new).cpu().numpy()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    print("allocator: torch", flush=True)
    p = h.Problem(dp, allocator="torch", leaf_size=64, aca_tol=1e-7)
    held = torch.cuda.memory_allocated() - base
    got = p.eval(theta, dz)
    pred = p.predict(dz, new).cpu().numpy()          # adds prediction workspaces
    held_more = torch.cuda.memory_allocated() - base
    p.close()
    torch.cuda.synchronize()
    assert held > 1 << 20 and held_more >= held
    assert torch.cuda.memory_allocated() == base
    assert tuple(got) == tuple(ref)
    np.testing.assert_array_equal(pred, ref_pred)


def test_failing_allocator_gives_nomem_and_frees_everything():
    import torch
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_TESTS, 741)
    dp = _cuda(synth.uniform_points(2000, 2, rng))
    live = {}
    calls = [0]

    def make(limit):
        def _alloc(nbytes, stream, user):
            calls[0] += 1
            if calls[0] > limit:
                return None
            t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
            live[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, stream, user):
            del live[int(ptr)]
        return h.Allocator(h.ALLOC_FN(_alloc), h.FREE_FN(_free), None)

    for limit in (0, 5, 40):
        calls[0] = 0
        a = make(limit)
        out = ctypes.c_void_p()
        print(f"failing allocator after {limit} blocks", flush=True)
        st = h.lib().hmle_build_tree_alloc(h._ptr(dp), 2000, 2, ctypes.byref(h.make_opts(leaf_size=64)),
                                           ctypes.byref(a), h._stream(), ctypes.byref(out))
        assert st == h.HMLE_E_NOMEM, st
        assert out.value is None
        assert b"returned NULL" in h.lib().hmle_last_error(None)
        assert not live, len(live)
    # a working allocator of the same kind builds and releases everything
    calls[0] = 0
    a = make(10 ** 9)
    with h.Problem(dp, allocator=a, leaf_size=64) as p:
        assert len(live) > 10
        p.eval((1.0, 0.1, 0.5, 0.01), _cuda(np.ones(2000)))
    assert not live


def test_allocator_without_free_is_refused():
    import paper_2104_07146_amd as h
    dp = _cuda(np.random.default_rng(0).random((10, 2)))
    a = h.Allocator(h.ALLOC_FN(lambda n, s, u: None), h.FREE_FN(), None)
    out = ctypes.c_void_p()
    st = h.lib().hmle_build_tree_alloc(h._ptr(dp), 10, 2, None, ctypes.byref(a), h._stream(), ctypes.byref(out))
    assert st == h.HMLE_E_INVALID
