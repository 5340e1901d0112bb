"""GPU: the batched form (many chains sharing launches of the sweep kernel).

Chains of a batch share launches (each chain with its own p-side group and
z-pass blocks), so the order in which a chain sums X^T z depends on its share
of blocks: a batch chain is held to the oracle's parity bars sweep by sweep
(as a lone sampler is), and two identical batches must agree bit for bit.
Datasets span the one-block path (p <= 16), the tiled path and bfloat16
storage (checked against the oracle on the bfloat16-rounded design).
"""
import numpy as np
import pytest

import synth
from gpu_util import b_scale, dataset, need_gpu, z_scale

pytestmark = pytest.mark.gpu

SETS = [((3001, 12, 61), "f32", 2), ((2051, 257, 62), "f32", 2), ((1500, 130, 63), "bf16", 1),
        ((4000, 64, 64), "bf16", 1), ((2500, 20, 65), "f32", 1)]


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def beta_tol(G, lam, tau, Xf, z, beta):
    Qi = np.abs(np.linalg.inv(G + tau * np.diag(lam)))
    return Qi @ (1e-5 * b_scale(Xf, z)) + 1e-10 * np.abs(beta)


def make_batch(env, sets, **kw):
    torch, hsp = env
    ds = [(dataset(*shape), xt, c) for shape, xt, c in sets]
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), xt) for d, xt, _ in ds]
    return ds, hsp.Batch(datasets, [c for _, _, c in ds], **kw)


def test_batch_chains_follow_the_oracle(env, orc):
    ds, b = make_batch(env, SETS, seed=9, chain_id=3, debug_store_z=True)
    assert len(b) == sum(c for _, _, c in SETS)
    ors = []
    cid = 3
    for d, xt, c in ds:
        if xt == "bf16":
            Xo = synth.bf16_bits(d.X).reshape(d.X.shape)
            Xf = synth.bf16_to_f32(Xo).reshape(d.X.shape)
        else:
            Xo = Xf = d.X
        G = orc.gram(Xo)
        for _ in range(c):
            ors.append((Xo, Xf, d.y, G, orc.Chain(d.p), cid))
            cid += 1
    for k in range(1, 4):
        b.sweep(1)
        b.sync()
        for i, (Xo, Xf, y, G, ch, cid) in enumerate(ors):
            beta_prev = ch.beta.copy()
            zo, bo, _ = ch.sweep_once(Xo, y, G, seed=9, chain=cid, want_z=True)
            z, att, bg = b.chain(i).debug()
            assert np.all(z * (2.0 * y - 1.0) > 0), (k, i)
            assert np.max(np.abs(z - zo) / z_scale(Xf, beta_prev)) < 1e-5, (k, i)
            g = b.chain(i).state()
            assert g["sweep"] == ch.sweep == k
            tol = beta_tol(G, ch.lam_m2, ch.tau_m2, Xf, zo, ch.beta) * 10
            assert np.all(np.abs(g["beta"] - ch.beta) <= tol), (k, i)
            for key, ref in [("lam_m2", ch.lam_m2), ("nu_m1", ch.nu_m1)]:
                np.testing.assert_allclose(g[key], ref, rtol=1e-4)
            assert g["tau_m2"] == pytest.approx(ch.tau_m2, rel=1e-4)
            assert g["xi_m1"] == pytest.approx(ch.xi_m1, rel=1e-4)
    b.close()


def test_batch_chain_equals_lone_chain(env):
    """A chain in a pack (its own group and z-block counts) draws bitwise what
    the same chain draws alone: X^T z is exact in any split of the rows, and
    the p-side's arithmetic does not depend on its group size."""
    torch, hsp = env
    ds, b = make_batch(env, SETS, seed=4, chain_id=5, record_lambda=True)
    b.sweep(4)
    b.sync()
    batch = [b.chain(i).draws() for i in range(len(b))]
    b.close()
    i = 0
    for d, xt, c in ds:
        for _ in range(c):
            s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=4,
                            chain_id=5 + i, x_type=xt, record_lambda=True)
            s.sweep(4)
            s.sync()
            bb, tb, lb, nb = batch[i]
            bl, tl, ll, nl = s.draws()
            s.close()
            assert nb == nl == 4
            assert np.array_equal(bb, bl) and np.array_equal(tb, tl) and np.array_equal(lb, ll), (i, d.p, xt)
            i += 1


def test_batch_mixed_tile_heights_equal_lone_chains(env):
    """Float32 chains with p <= 256 (32-row z tiles), 257 <= p <= 512 (16
    rows), 513 <= p <= 1024 (8 rows) and p > 1024 (4 rows) in one batch, with
    bfloat16 chains: each pack keeps one tile height, so every chain still
    draws bitwise what it draws alone."""
    torch, hsp = env
    sets = [((2003, 1000, 66), "f32", 1), ((2003, 1100, 67), "f32", 1), ((1500, 300, 68), "f32", 1),
            ((1500, 2100, 69), "bf16", 1), ((1800, 700, 70), "bf16", 1), ((2222, 150, 71), "f32", 1)]
    ds, b = make_batch(env, sets, seed=6, chain_id=2)
    b.sweep(3)
    b.sync()
    batch = [b.chain(i).draws() for i in range(len(b))]
    b.close()
    for i, (d, xt, _) in enumerate(ds):
        s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=6,
                        chain_id=2 + i, x_type=xt)
        s.sweep(3)
        bl, tl, nl = s.draws()
        s.close()
        bb, tb, nb = batch[i]
        assert nb == nl == 3
        assert np.array_equal(bb, bl) and np.array_equal(tb, tl), (i, d.p, xt)


def test_batch_is_reproducible(env):
    outs = []
    for _ in range(2):
        _, b = make_batch(env, SETS, seed=4, record_lambda=True)
        b.sweep(4)
        b.sync()
        outs.append([b.chain(i).draws() for i in range(len(b))])
        b.close()
    for (b1, t1, l1, n1), (b2, t2, l2, n2) in zip(*outs):
        assert n1 == n2 == 4
        assert np.array_equal(b1, b2) and np.array_equal(t1, t2) and np.array_equal(l1, l2)


def test_batch_many_chains_on_shared_data(env):
    torch, hsp = env
    d = dataset(5000, 150, 65)
    b = hsp.Batch([(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda())], 16, seed=5)
    b.sweep(3)
    b.sweep(2)
    b.sync()
    betas = np.stack([b.chain(i).state()["beta"] for i in range(16)])
    assert np.all(np.isfinite(betas)) and len({betas[i].tobytes() for i in range(16)}) == 16
    assert all(b.chain(i).state()["sweep"] == 5 for i in range(16))
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
        # the recovered sign of the large leading coefficient (4.0)
        assert st["beta"][1] > 0
    b.close()


# ---- the multi-chain z pass (chains sharing a bfloat16 design) ----------------------
def _flip_aware(orc, Xo, Xf, y, z, att, b, zo, ao, bo_branch, beta_prev):
    """z on rows without a flip, and X^T z with the flipped rows' share in the bar."""
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo_branch == 1))
    assert flips.sum() <= max(1, int(1e-5 * y.size))
    ok = ~flips
    assert np.max(np.abs(z[ok] - zo[ok]) / z_scale(Xf[ok], beta_prev)) < 1e-5
    dz = np.abs(z.astype(np.float64) - zo)
    dz[ok] = 0.0
    slack = np.abs(Xf[flips].astype(np.float64)).T @ dz[flips] if flips.any() else 0.0
    assert np.all(np.abs(b - orc.xtz(Xo, zo)) <= 1e-5 * b_scale(Xf, zo) + slack)


@pytest.mark.parametrize("sets", [
    [((3001, 1000, 71), "bf16", 16)],
    [((5003, 200, 72), "bf16", 3), ((2500, 12, 73), "bf16", 2), ((1777, 1024, 74), "bf16", 2),
     ((3001, 40, 75), "f32", 2)],
])
def test_multi_chain_pass_follows_the_oracle(env, orc, sets):
    """Every chain of a multi-chain pass, sweep by sweep, against the oracle
    on the bfloat16-rounded design: z and X^T z to the 1e-5 bars, beta to the
    propagated bar, the hyperparameters to 1e-4."""
    ds, b = make_batch(env, sets, seed=12, chain_id=7, debug_store_z=True)
    ors = []
    cid = 7
    for d, xt, c in ds:
        if xt == "bf16":
            Xo = synth.bf16_bits(d.X).reshape(d.X.shape)
            Xf = synth.bf16_to_f32(Xo).reshape(d.X.shape)
        else:
            Xo = Xf = d.X
        G = orc.gram(Xo)
        for _ in range(c):
            ors.append((Xo, Xf, d.y, G, orc.Chain(d.p), cid))
            cid += 1
    for k in range(1, 3):
        b.sweep(1)
        b.sync()
        for i, (Xo, Xf, y, G, ch, cid) in enumerate(ors):
            beta_prev = ch.beta.copy()
            zo, ao, bro = orc.z_step(Xo, y, beta_prev, 12, k, chain=cid)
            zo2, bo, _ = ch.sweep_once(Xo, y, G, seed=12, chain=cid, want_z=True)
            assert np.array_equal(zo, zo2)
            z, att, bg = b.chain(i).debug()
            assert np.all(z * (2.0 * y - 1.0) > 0), (k, i)
            _flip_aware(orc, Xo, Xf, y, z, att, bg, zo, ao, bro, beta_prev)
            g = b.chain(i).state()
            assert g["sweep"] == ch.sweep == k
            tol = beta_tol(G, ch.lam_m2, ch.tau_m2, Xf, zo, ch.beta) * 10
            assert np.all(np.abs(g["beta"] - ch.beta) <= tol), (k, i)
            for key, ref in [("lam_m2", ch.lam_m2), ("nu_m1", ch.nu_m1)]:
                np.testing.assert_allclose(g[key], ref, rtol=1e-4)
            assert g["tau_m2"] == pytest.approx(ch.tau_m2, rel=1e-4)
    b.close()


def test_multi_chain_pass_is_reproducible(env):
    sets = [((4099, 300, 76), "bf16", 5), ((2051, 16, 77), "bf16", 3)]
    outs = []
    for _ in range(2):
        _, b = make_batch(env, sets, seed=13, record_lambda=True)
        b.sweep(5)
        b.sync()
        outs.append([b.chain(i).draws() for i in range(len(b))])
        b.close()
    for (b1, t1, l1, n1), (b2, t2, l2, n2) in zip(*outs):
        assert n1 == n2 == 5
        assert np.array_equal(b1, b2) and np.array_equal(t1, t2) and np.array_equal(l1, l2)


def test_multi_chain_off_equals_lone_chains(env):
    """With the multi-chain pass switched off, chains on a shared bfloat16
    design draw bitwise what lone samplers draw."""
    torch, hsp = env
    sets = [((3001, 150, 78), "bf16", 3)]
    ds, b = make_batch(env, sets, seed=14, chain_id=4, multi_chain_z=False)
    b.sweep(3)
    b.sync()
    batch = [b.chain(i).draws() for i in range(len(b))]
    b.close()
    d, xt, _ = ds[0]
    for i in range(3):
        s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=14,
                        chain_id=4 + i, x_type=xt)
        s.sweep(3)
        bl, tl, _ = s.draws()
        s.close()
        assert np.array_equal(batch[i][0], bl) and np.array_equal(batch[i][1], tl)


@pytest.mark.parametrize("pre", [0, 8, 32])
def test_factorisation_beside_the_pass_changes_nothing(env, pre):
    """Chains of a multi-chain pass may draw lambda, tau, nu, xi and factor Q
    in a launch beside the pass (p > 16) and take b after it: the same
    arithmetic as one launch after the pass, so every draw is bitwise the
    same for any number of blocks per chain, or with no such launch."""
    sets = [((3001, 1000, 71), "bf16", 4), ((2500, 12, 73), "bf16", 2), ((2051, 257, 62), "f32", 1),
            ((1777, 130, 74), "bf16", 3)]
    outs = {}
    for blocks in (16, pre):
        _, b = make_batch(env, sets, seed=17, chain_id=1, record_lambda=True)
        b.set_shape(64, blocks)
        b.sweep(3)
        b.sync()
        outs[blocks] = [b.chain(i).draws() for i in range(len(b))]
        b.close()
    for i, (x, y) in enumerate(zip(outs[16], outs[pre])):
        assert x[3] == y[3] == 3
        assert all(np.array_equal(u, v) for u, v in zip(x[:3], y[:3])), (i, pre)
