"""GPU: one batched sweep of the benchmark's whole composition against the oracle.

64 uneven float32 datasets (one chain each) and 16 chains on the N = 1e6,
p = 1000 design stored in bfloat16, batched as the benchmark batches them (the
16 chains share one read of X per sweep on the matrix cores; the others take
their z passes from shared queues; the launches run on two streams).  Every
one of the 16 shared-design chains and 4 of the uneven chains (the longest,
the widest, one of 32-row and one of 16-row z tiles) starts from a state of
its own with realistic |x_i beta|; after one batched sweep each is held to
one oracle sweep from the same state (Section 5, z and beta steps; Eq. 12):
z on every row and X^T z at the 1e-5 bars (rows whose accepted proposal or
branch differs are counted and bounded, and enter the X^T z bar with their
share), beta at the propagated bar, lambda, nu, tau and xi at 1e-4.  The
shared-design chains are checked on the bfloat16-rounded design.
"""
import numpy as np
import pytest

import synth
from gpu_util import need_gpu

pytestmark = pytest.mark.gpu

SEED, CID0, SWEEP0 = 23, 100, 7


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def start_state(d, k):
    """A state near the truth: |x_i beta| of the size the chain reaches."""
    rng = np.random.default_rng(500 + k)
    return dict(beta=d.beta_true + rng.normal(0, 0.02, d.p), lam_m2=rng.gamma(2.0, 1.0, d.p),
                nu_m1=rng.gamma(2.0, 1.0, d.p), tau_m2=float(rng.gamma(3.0, 1.0)),
                xi_m1=float(rng.gamma(2.0, 1.0)))


def test_benchmark_batch_one_sweep_against_oracle(env, orc):
    torch, hsp = env
    shapes = synth.batch_shapes(64, seed=1000)
    ds = [synth.batch_dataset(k, N, p) for k, (N, p) in enumerate(shapes)]
    beta_true, _ = synth.sparse_beta(1000, 10, 13)
    big = synth.probit_design(1_000_000, 1000, beta_true, 13, True, "n1000000_p1000")
    datasets = [(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), "f32") for d in ds]
    datasets.append((torch.from_numpy(big.X).cuda(), torch.from_numpy(big.y).cuda(), "bf16"))
    b = hsp.Batch(datasets, [1] * len(ds) + [16], seed=SEED, chain_id=CID0, max_draws=8, debug_store_z=True)
    del datasets
    torch.cuda.empty_cache()

    Ns = np.array([N for N, _ in shapes])
    ps = np.array([p for _, p in shapes])
    uneven = {int(np.argmax(Ns)), int(np.argmax(ps)), int(np.flatnonzero(ps <= 256)[0]),
              int(np.flatnonzero((ps > 256) & (ps <= 512))[-1])}
    checked = sorted(uneven) + list(range(64, 80))
    states = {}
    for i in checked:
        d = ds[i] if i < 64 else big
        st = start_state(d, i)
        b.chain(i).set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], SWEEP0)
        states[i] = st
    b.sweep(1)
    b.sync()

    bits = synth.bf16_bits(big.X).reshape(big.X.shape)
    Xbf = synth.bf16_to_f32(bits).reshape(big.X.shape)
    G_big = orc.gram_fast(bits)
    abs_big = np.abs(Xbf)  # float32 |X|: only sets the tolerance scales
    for i in checked:
        if i < 64:
            d = ds[i]
            Xo = Xf = d.X
            y, G, absX = d.y, orc.gram_fast(d.X), np.abs(d.X)
        else:
            Xo, Xf, y, G, absX = bits, Xbf, big.y, G_big, abs_big
        st = states[i]
        cid = CID0 + i
        ch = orc.Chain(G.shape[0], st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], SWEEP0)
        zo, ao, bro = orc.z_step(Xo, y, st["beta"], SEED, SWEEP0 + 1, chain=cid)
        zo2, bo, _ = ch.sweep_once(Xo, y, G, seed=SEED, chain=cid, want_z=True)
        assert np.array_equal(zo, zo2)
        z, att, bg = b.chain(i).debug()
        assert np.all(z * (2.0 * y - 1.0) > 0), i
        # z on every row without a flipped proposal or branch
        flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bro == 1))
        assert flips.sum() <= max(1, int(1e-5 * y.size)), (i, int(flips.sum()))
        ok = ~flips
        zs = np.maximum(absX @ np.abs(st["beta"]).astype(np.float32), 1.0)
        assert np.max(np.abs(z[ok] - zo[ok]) / zs[ok]) < 1e-5, i
        # X^T z: of the kernel's own z, and the oracle's with the flipped rows' share
        bs_own = absX.T @ np.abs(z).astype(np.float32)
        assert np.max(np.abs(bg - orc.xtz(Xo, z.astype(np.float64))) / bs_own) < 1e-5, i
        dz = np.abs(z.astype(np.float64) - zo)
        dz[ok] = 0.0
        slack = absX[flips].astype(np.float64).T @ dz[flips] if flips.any() else 0.0
        bs = absX.T @ np.abs(zo).astype(np.float32)
        assert np.all(np.abs(bg - bo) <= 1e-5 * bs + slack), i
        # the p-side from the same state
        g = b.chain(i).state()
        assert g["sweep"] == ch.sweep == SWEEP0 + 1
        Qi = np.abs(np.linalg.inv(G + ch.tau_m2 * np.diag(ch.lam_m2)))
        tol = (Qi @ (1e-5 * bs.astype(np.float64) + slack) + 1e-10 * np.abs(ch.beta)) * 10
        assert np.all(np.abs(g["beta"] - ch.beta) <= tol), i
        for key, ref in [("lam_m2", ch.lam_m2), ("nu_m1", ch.nu_m1)]:
            np.testing.assert_allclose(g[key], ref, rtol=1e-4)
        assert g["tau_m2"] == pytest.approx(ch.tau_m2, rel=1e-4)
        assert g["xi_m1"] == pytest.approx(ch.xi_m1, rel=1e-4)
    b.close()
