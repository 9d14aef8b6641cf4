"""GPU test of the schedule autotuner (hmle_autotune, coordinate search over
pair_chunk, sketch_group, seg_entries, gseg_rows and the sum_kc tile shape):
every distinct candidate is measured once, the first is the starting
schedule, each later one differs from an earlier one in one option, and the
returned schedule is the fastest measured. The options change only which
workgroup computes which products (so sums in another order and, at a
threshold, a truncation rank by one), so the log-likelihood with any of them
agrees with the default schedule far inside the H-approximation error, and
with the dense oracle to the small-n target. The JSON cache returns a stored
schedule without measuring and stores a measured one."""
import json

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("pair_chunk", "sketch_group", "seg_entries", "gseg_rows", "sum_kc")


def _problem():
    import torch
    from oracle import dense
    rng = synth.rng_for(synth.W_TESTS, 700)
    n = 3000
    pts = synth.uniform_points(n, 2, rng)
    theta = (1.0, 0.1, 0.5, 0.01)
    z = dense.sample(pts, theta, synth.standard_normal(n, rng))
    return pts, theta, z, torch.tensor(pts, device="cuda"), torch.tensor(z, device="cuda")


def test_autotune_search_and_agreement():
    import paper_2104_07146_amd as h
    from oracle import dense
    pts, theta, z, dp, zc = _problem()
    print("autotune n=3000", flush=True)
    best, tried = h.autotune(dp, theta, leaf_size=64, aca_tol=1e-6)
    keys = [tuple(s[k] for k in KEYS) for s, _ in tried]
    assert len(set(keys)) == len(keys) and 1 <= len(keys) <= 25
    assert keys[0] == (1, 8, 8, 512, 16)                 # the defaults start the search
    for i in range(1, len(keys)):
        assert any(sum(a != b for a, b in zip(keys[i], keys[j])) == 1 for j in range(i)), keys[i]
    assert all(ms > 0 for _, ms in tried)
    assert tuple(best[k] for k in KEYS) in keys
    assert min(ms for _, ms in tried) == [ms for s, ms in tried if s == best][0]
    with h.Problem(dp, leaf_size=64, aca_tol=1e-6) as p:
        a = p.eval(theta, zc)
    with h.Problem(dp, leaf_size=64, aca_tol=1e-6, **best) as p:
        b = p.eval(theta, zc)
    for sched in [dict(pair_chunk=4, sketch_group=2), dict(sketch_group=16, seg_entries=4),
                  dict(seg_entries=16, gseg_rows=256), dict(gseg_rows=1024, sum_kc=32), dict(sum_kc=32)]:
        with h.Problem(dp, leaf_size=64, aca_tol=1e-6, **sched) as p:
            c = p.eval(theta, zc)
        assert abs(c[0] - a[0]) <= 1e-8 * abs(a[0]), (sched, c[0], a[0])
    assert abs(b[0] - a[0]) <= 1e-8 * abs(a[0])
    ref = dense.loglik(pts, z, theta)
    assert abs(b[0] - ref[0]) <= 1e-6 * abs(ref[0])


def test_tuned_schedule_cache(tmp_path):
    import paper_2104_07146_amd as h
    pts, theta, z, dp, zc = _problem()
    path = str(tmp_path / "tuned.json")
    key = h.tune_key(dp.shape[0], dp.shape[1], leaf_size=64, aca_tol=1e-6)
    stored = {"pair_chunk": 2, "sketch_group": 4, "seg_entries": 16, "gseg_rows": 256, "sum_kc": 32}
    with open(path, "w") as f:
        json.dump({key: {"schedule": stored}}, f)
    assert h.tuned_schedule(dp, theta, path=path, leaf_size=64, aca_tol=1e-6) == stored
    # another configuration is missing: not tuned on request, else tuned and stored
    assert h.tuned_schedule(dp, theta, path=path, tune_if_missing=False, leaf_size=32, aca_tol=1e-6) is None
    got = h.tuned_schedule(dp[:1500], theta, path=path, leaf_size=32, aca_tol=1e-6)
    with open(path) as f:
        cache = json.load(f)
    assert len(cache) == 2 and key in cache
    key2 = h.tune_key(1500, 2, leaf_size=32, aca_tol=1e-6)
    assert cache[key2]["schedule"] == got
