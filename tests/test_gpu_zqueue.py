"""GPU: packs whose chains take their z passes from one shared queue.

The queue's worker blocks take units of rows of any chain of the pack and
add their float64 tile sums of x_ij z_i into that chain's accumulator of
X^T z (Section 5, z step and beta step vi).  The tile sums lie on a fixed
grid on which every one of those additions is exact, so a chain's draws may
not depend on which worker took which unit, nor on the unit size: these
tests hold that bitwise, against the same batch with z-pass blocks per
chain, for units from one row tile to a whole chain, and against lone
samplers.  The sets span chains shorter than one unit, the one-block p-side
(p <= 16), one and two 16-byte vectors per lane, bfloat16 storage, and more
chains than a wave has lanes (the workers' search for the chain with most
units left).
"""
import numpy as np
import pytest

from gpu_util import dataset, need_gpu

pytestmark = pytest.mark.gpu

SETS = [((37, 20, 81), "f32", 2), ((3001, 12, 82), "f32", 3), ((2051, 257, 83), "f32", 2),
        ((1500, 130, 84), "bf16", 1), ((4000, 64, 85), "f32", 4), ((999, 500, 86), "f32", 1),
        ((2500, 96, 87), "f32", 60)]
SWEEPS = 3


@pytest.fixture(scope="module")
def env():
    return need_gpu()


@pytest.fixture(scope="module")
def data():
    return [(dataset(*shape), xt, c) for shape, xt, c in SETS]


def run_batch(env, data, kib):
    torch, hsp = env
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), xt) for d, xt, _ in data]
    b = hsp.Batch(datasets, [c for _, _, c in data], seed=21, chain_id=7, record_lambda=True)
    if kib is not None:
        b.set_shape(kib, 16)
        assert b.plan()[3] == f"zq={kib} pre=16 (set)"
    b.sweep(SWEEPS)
    b.sync()
    out = [b.chain(i).draws() for i in range(len(b))]
    states = [b.chain(i).state()["sweep"] for i in range(len(b))]
    b.close()
    assert states == [SWEEPS] * len(out)
    return out


@pytest.fixture(scope="module")
def queued(env, data):
    return run_batch(env, data, 64)


def same(x, y):
    return all(np.array_equal(u, v) for u, v in zip(x[:3], y[:3])) and x[3] == y[3]


@pytest.mark.parametrize("kib", [0, 1, 4096, None])
def test_queue_unit_sizes_and_blocks_per_chain_agree(env, data, queued, kib):
    """kib = 0: every chain with z blocks of its own; 1: units of one or two
    row tiles; 4096: one unit per chain; None: the built-in plan."""
    other = run_batch(env, data, kib)
    assert len(other) == len(queued) == sum(c for _, _, c in SETS)
    for i, (x, y) in enumerate(zip(queued, other)):
        assert x[3] == SWEEPS
        assert same(x, y), (i, kib)


def test_queue_chains_equal_lone_chains(env, data, queued):
    torch, hsp = env
    i = 0
    for d, xt, c in data:
        s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=21,
                        chain_id=7 + i, x_type=xt, record_lambda=True)
        s.sweep(SWEEPS)
        s.sync()
        lone = s.draws()
        s.close()
        assert same(queued[i], lone), (i, d.N, d.p, xt)
        i += c


def test_queue_setting_is_checked(env, data):
    torch, hsp = env
    d, xt, _ = data[1]
    b = hsp.Batch([(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), xt)], 2, seed=1)
    for bad in ((-1, 16), (4097, 16), (64, -1), (64, 4097)):
        with pytest.raises(hsp.HspError) as e:
            b.set_shape(*bad)
        assert e.value.code == hsp.HSP_EINVAL
    b.close()
