"""GPU: the autotuner changes how the sweep kernel splits its work, never what
it draws.  A measured plan and a plan forced through the cache file draw, bit
for bit, what the built-in plan draws."""
import os

import numpy as np
import pytest

from gpu_util import dataset, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def _run(torch, hsp, d, n, **kw):
    s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=21, max_draws=n, **kw)
    plan = s.plan()
    s.sweep(n)
    betas, taus, _ = s.draws()
    s.close()
    return plan, betas, taus


@pytest.mark.parametrize("N,p,xt", [(100003, 300, "f32"), (60001, 10, "f32"), (80021, 130, "bf16")])
def test_measured_plan_draws_what_the_default_draws(env, N, p, xt, tmp_path, monkeypatch):
    torch, hsp = env
    monkeypatch.setenv("HSP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    d = dataset(N, p, 700 + p)
    p0, b0, t0 = _run(torch, hsp, d, 25, x_type=xt)
    p1, b1, t1 = _run(torch, hsp, d, 25, x_type=xt, autotune=True)
    assert p0[4] == "built-in" and p1[4].endswith("(measured)"), (p0, p1)
    assert np.array_equal(b0, b1) and np.array_equal(t0, t1), (p0, p1)
    # the choice went into the cache, and a new state takes it from there
    p2, b2, _ = _run(torch, hsp, d, 25, x_type=xt, autotune=True)
    assert p2[4].endswith("(cache)") and p2[:4] == p1[:4], (p1, p2)
    assert np.array_equal(b0, b2)


def test_cached_plan_far_from_default_draws_the_same(env, tmp_path, monkeypatch):
    torch, hsp = env
    path = str(tmp_path / "tune.txt")
    monkeypatch.setenv("HSP_TUNE_CACHE", path)
    d = dataset(50021, 257, 731)
    p0, b0, t0 = _run(torch, hsp, d, 20)
    probe = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=21)
    key = hsp.hsp_tune_key(probe.h)
    probe.close()
    for value in ["gp=2 pct=0 unit=1", "gp=7 pct=100 unit=64", "gp=1 pct=13 unit=5"]:
        hsp.hsp_tune_cache_put(path, key, value)
        p1, b1, t1 = _run(torch, hsp, d, 20, autotune=True)
        assert p1[4] == value + " (cache)", p1
        assert p1[0] == int(value.split()[0][3:]) and p1[0] != p0[0]
        assert np.array_equal(b0, b1) and np.array_equal(t0, t1), value
    # an entry the state cannot use is measured over instead
    hsp.hsp_tune_cache_put(path, key, "gp=0 pct=40 unit=8")
    p2, b2, _ = _run(torch, hsp, d, 20, autotune=True)
    assert p2[4].endswith("(measured)")
    assert np.array_equal(b0, b2)


def _batch_draws(torch, hsp, ds, counts, n, **kw):
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), xt) for d, xt in ds]
    b = hsp.Batch(datasets, counts, seed=5, max_draws=n, **kw)
    b.sweep(n)
    b.sync()
    plan = b.plan()
    out = [c.draws()[0] for c in b.chains]
    b.close()
    return plan, out


def test_tuned_batch_draws_what_the_default_batch_draws(env, tmp_path, monkeypatch):
    """Packs of float32 chains and a multi-chain z pass over a shared
    bfloat16 design, tuned by measurement and then from the cache."""
    torch, hsp = env
    monkeypatch.setenv("HSP_TUNE_CACHE", str(tmp_path / "tune.txt"))
    ds = [(dataset(20011, 40, 741), "f32"), (dataset(9001, 130, 742), "f32"), (dataset(60013, 200, 743), "bf16")]
    counts = [1, 2, 5]
    p0, d0 = _batch_draws(torch, hsp, ds, counts, 12)
    p1, d1 = _batch_draws(torch, hsp, ds, counts, 12, autotune=True)
    assert p0[3] == "built-in" and p1[3].endswith("(measured)"), (p0, p1)
    for a, b in zip(d0, d1):
        assert np.array_equal(a, b), (p0, p1)
    p2, d2 = _batch_draws(torch, hsp, ds, counts, 12, autotune=True)
    assert p2[3].endswith("(cache)") and p2[:2] == p1[:2], (p1, p2)
    for a, b in zip(d0, d2):
        assert np.array_equal(a, b)
