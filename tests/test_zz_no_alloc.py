"""The allocation-free variogram call (hmle_variogram_noalloc) against the
allocating one (hmle_variogram), through the C ABI.

Both run the same kernels in the same fixed summation order, so the features
must agree bit for bit. Two calls in a row (the second smaller) check that the
fixed workspace carries nothing from one call into the next; a call larger
than the workspace must be refused before anything is launched. The features
themselves are checked against the oracle as for the allocating call.
"""
import ctypes

import numpy as np
import pytest

import synth
from oracle import learned

pytestmark = pytest.mark.gpu


def _cuda(a, dtype=np.float64):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _fields(rng, sizes, dim):
    pts = [rng.random((n, dim)) for n in sizes]
    zs = [rng.standard_normal(n) for n in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return pts, zs, off


def _raw_call(fn, dp, dz, off, dim, out, sel=None, soff=None):
    import torch
    import paper_2104_07146_amd as h
    return fn(h._ptr(dp), h._ptr(dz), off.ctypes.data, len(off) - 1, dim,
              None if sel is None else h._fptr(sel, "int32"), None if soff is None else soff.ctypes.data,
              torch.cuda.current_stream().cuda_stream, h._fptr(out))


@pytest.mark.parametrize("dim", [2, 3])
def test_noalloc_equals_allocating_call_two_calls_in_a_row(dim):
    import torch
    import paper_2104_07146_amd as h
    L = h.lib()
    rng = synth.rng_for(synth.W_LEARNED, 70 + dim)
    for call, sizes in enumerate([[1000, 129, 4096, 2, 777], [300, 1]]):
        pts, zs, off = _fields(rng, sizes, dim)
        dp, dz = _cuda(np.concatenate(pts)), _cuda(np.concatenate(zs))
        print(f"noalloc variogram dim={dim} call={call} sizes={sizes}", flush=True)
        want = torch.full((len(sizes), h.N_FEAT), np.nan, dtype=torch.float32, device="cuda")
        got = torch.full((len(sizes), h.N_FEAT), np.nan, dtype=torch.float32, device="cuda")
        assert _raw_call(L.hmle_variogram, dp, dz, off, dim, want) == h.HMLE_OK
        assert _raw_call(L.hmle_variogram_noalloc, dp, dz, off, dim, got) == h.HMLE_OK
        w, g = want.cpu().numpy(), got.cpu().numpy()
        np.testing.assert_array_equal(g, w)
        for q, n in enumerate(sizes):
            ref = learned.variogram_features(pts[q], zs[q])
            err = np.abs(g[q] - ref) / np.maximum(1.0, np.abs(ref))
            assert float(err.max()) <= 1e-6, (call, q, n)


def test_noalloc_with_point_subsets():
    import torch
    import paper_2104_07146_amd as h
    rng = synth.rng_for(synth.W_LEARNED, 80)
    sizes = [9000, 3000]
    pts, zs, off = _fields(rng, sizes, 2)
    sel = [synth.subset_indices(n, 2048, rng) for n in sizes]
    soff = np.array([0, 2048, 4096], dtype=np.int64)
    dp, dz, dsel = _cuda(np.concatenate(pts)), _cuda(np.concatenate(zs)), _cuda(np.concatenate(sel), np.int32)
    print("noalloc variogram with subsets", flush=True)
    want = h.variogram(dp, dz, off, dsel, soff).cpu().numpy()
    got = h.variogram(dp, dz, off, dsel, soff, noalloc=True).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    # a smaller call right after: one field, no subset
    pts2, zs2, off2 = _fields(rng, [513], 2)
    want2 = h.variogram(_cuda(pts2[0]), _cuda(zs2[0]), off2).cpu().numpy()
    got2 = h.variogram(_cuda(pts2[0]), _cuda(zs2[0]), off2, noalloc=True).cpu().numpy()
    np.testing.assert_array_equal(got2, want2)


def test_noalloc_refuses_a_call_beyond_its_workspace():
    import torch
    import paper_2104_07146_amd as h
    L = h.lib()
    # 63 fields of 4096 points need 63 * 528 tiles * 512 bytes + offsets > 16 MiB
    count, m = 63, 4096
    rng = synth.rng_for(synth.W_LEARNED, 90)
    dp = _cuda(rng.random((count * m, 2)))
    dz = _cuda(rng.standard_normal(count * m))
    off = (np.arange(count + 1) * m).astype(np.int64)
    out = torch.full((count, h.N_FEAT), 7.0, dtype=torch.float32, device="cuda")
    print("noalloc variogram oversize refusal", flush=True)
    st = _raw_call(L.hmle_variogram_noalloc, dp, dz, off, 2, out)
    assert st == h.HMLE_E_INVALID
    assert b"workspace" in L.hmle_last_error(None)
    assert bool((out == 7.0).all())           # nothing was written
    # 62 such fields fit, and agree with the allocating call
    off62 = off[:63]
    want = torch.empty((62, h.N_FEAT), dtype=torch.float32, device="cuda")
    got = torch.empty((62, h.N_FEAT), dtype=torch.float32, device="cuda")
    assert _raw_call(L.hmle_variogram, dp, dz, off62, 2, want) == h.HMLE_OK
    assert _raw_call(L.hmle_variogram_noalloc, dp, dz, off62, 2, got) == h.HMLE_OK
    np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())
