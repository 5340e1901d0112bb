"""GPU: the batched form (many chains, one graph replay per sweep).

A batch must be exactly the set of its chains run alone: chain i of a batch
uses counter chain id chain_id + i, shares its dataset's X, y and G, and
draws bit for bit what a lone sampler with that chain id draws.  Datasets
span the one-block path (p <= 128), the tiled path and bfloat16 storage.
"""
import numpy as np
import pytest

import synth
from gpu_util import dataset, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def lone(env, d, x_type, seed, chain_id, n):
    torch, hsp = env
    s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=seed,
                    chain_id=chain_id, x_type=x_type, record_lambda=True)
    s.sweep(n)
    out = s.draws()
    st = s.state()
    s.close()
    return out, st


def test_batch_chains_equal_lone_samplers(env):
    torch, hsp = env
    sets = [(dataset(3001, 20, 61), "f32", 2), (dataset(2051, 257, 62), "f32", 2),
            (dataset(1500, 130, 63), "bf16", 1), (dataset(4000, 64, 64), "bf16", 1)]
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), xt) for d, xt, _ in sets]
    b = hsp.Batch(datasets, [c for _, _, c in sets], seed=9, chain_id=3, record_lambda=True)
    assert len(b) == 6
    b.sweep(4)
    b.sync()
    i = 0
    for d, xt, c in sets:
        for _ in range(c):
            (beta, tau, lam, n), st = lone(env, d, xt, 9, 3 + i, 4)
            bb, bt, bl, bn = b.chain(i).draws()
            assert n == bn == 4
            assert np.array_equal(beta, bb) and np.array_equal(tau, bt) and np.array_equal(lam, bl)
            sb = b.chain(i).state()
            for key in ("beta", "lam_m2", "nu_m1"):
                assert np.array_equal(st[key], sb[key])
            assert st["tau_m2"] == sb["tau_m2"] and st["xi_m1"] == sb["xi_m1"] and sb["sweep"] == 4
            i += 1
    # chains on the same data differ (their own counters)
    assert not np.array_equal(b.chain(0).state()["beta"], b.chain(1).state()["beta"])
    b.close()


def test_batch_many_chains_on_shared_data_and_more_sweeps(env):
    torch, hsp = env
    d = dataset(5000, 150, 65)
    b = hsp.Batch([(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda())], 16, seed=5)
    b.sweep(3)
    b.sweep(2)
    b.sync()
    betas = np.stack([b.chain(i).state()["beta"] for i in range(16)])
    assert np.all(np.isfinite(betas)) and len({betas[i].tobytes() for i in range(16)}) == 16
    (beta, tau, _, n), st = lone(env, d, "f32", 5, 11, 5)
    assert np.array_equal(st["beta"], betas[11])
    # a batch's chain cannot be destroyed on its own
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_destroy(b.chain(2).h)
    assert e.value.code == hsp.HSP_EINVAL
    b.close()


def test_batch_uneven_datasets(env):
    """A small version of the uneven-dataset batch: log-uniform N, uniform p."""
    torch, hsp = env
    shapes = synth.batch_shapes(6, seed=1000)
    shapes = [(max(2000, N // 20), p) for N, p in shapes]  # smaller N, same p mix
    ds = [synth.batch_dataset(k, N, p) for k, (N, p) in enumerate(shapes)]
    b = hsp.Batch([(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda()) for d in ds], 1, seed=2)
    b.set_timing(True)
    b.sweep(6)
    b.sync()
    ms, n = b.timing()
    assert n == 6 and ms > 0
    for i, d in enumerate(ds):
        st = b.chain(i).state()
        assert st["sweep"] == 6 and np.all(np.isfinite(st["beta"]))
    # the last dataset's chain equals its lone run
    (beta, _, _, _), st = lone(env, ds[-1], "f32", 2, len(ds) - 1, 6)
    assert np.array_equal(st["beta"], b.chain(len(ds) - 1).state()["beta"])
    b.close()
