"""GPU: long chains and the full-size workload.

* Long-chain parity: GPU chains and oracle chains with independent seeds must
  agree on the posterior mean and variance of every beta_j within
  4 sqrt(MCSE_gpu^2 + MCSE_oracle^2) (batch means, 20% burn-in), and the
  sign of each nonzero beta_true must be recovered (Section 6.1).
* Full size (N = 1,000,000, p = 1000, float32 X and bfloat16 X; the
  benchmark's launches): one z step and X^T z compared with the oracle on
  every row, G on sampled entries, and whole sweeps checked for the sign
  invariant and finiteness.

X^T z at full size is held to the oracle in two ways that hold whether or not
some row took another proposal than the oracle (a float32 vs float64
decision at a threshold): the GPU's b against the oracle's X^T z of the
GPU's own z (the product of X with the z the kernel drew), and against the
oracle's b with the flipped rows' difference |x_ij| |z_i - z_i'| added to
the bar.
"""
import math

import numpy as np
import pytest

import synth
from gpu_util import b_scale, need_gpu, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def batch_se(x):
    n = x.shape[0]
    nb = int(math.sqrt(n))
    m = n // nb
    bm = x[: nb * m].reshape(nb, m, *x.shape[1:]).mean(1)
    return bm.std(0, ddof=1) / math.sqrt(nb)


def pooled(chains):
    """Mean, variance and their batch-means standard errors over independent chains."""
    mus, vs, se_m, se_v = [], [], [], []
    for c in chains:
        mus.append(c.mean(0))
        se_m.append(batch_se(c))
    mu = np.mean(mus, 0)
    for c in chains:
        sq = (c - mu) ** 2
        vs.append(sq.mean(0))
        se_v.append(batch_se(sq))
    k = len(chains)
    return (mu, np.sqrt(np.sum(np.square(se_m), 0)) / k, np.mean(vs, 0),
            np.sqrt(np.sum(np.square(se_v), 0)) / k)


@pytest.mark.parametrize("which", ["n1000_p10", "n4000_p130", "n100000_p100", "n100000_p100_bf16"])
def test_long_chain_moments_agree_with_oracle(env, orc, which):
    """GPU and oracle chains with independent seeds: the same posterior moments
    within 4 MCSE.  The bfloat16 form is held to the oracle run on the
    bfloat16-rounded design (the posterior it targets)."""
    torch, hsp = env
    xt = "bf16" if which.endswith("bf16") else "f32"
    if which == "n1000_p10":
        d = synth.config1()
        n, chains = 3000, 4
    elif which == "n4000_p130":
        beta, _ = synth.sparse_beta(130, 5, 17, -2.0, 2.0)
        d = synth.probit_design(4000, 130, beta, 17, True)
        n, chains = 1500, 3
    else:
        # N = 1e5: from the cold start the large coefficients take ~400 sweeps
        # to settle (all of them together, through tau), so the burn-in is
        # longer than a fifth of the run
        d = synth.config2()
        n, chains = 2000, 3
    Xo = d.X if xt == "f32" else synth.bf16_bits(d.X).reshape(d.X.shape)
    burn = n // 5 if d.N < 100_000 else 600
    G = orc.gram(Xo)
    gpu, ora = [], []
    for c in range(chains):
        s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=101 + c,
                        max_draws=n, x_type=xt)
        s.sweep(n)
        b, _, _ = s.draws()
        gpu.append(b[burn:])
        s.close()
        ch = orc.Chain(d.p)
        bo, _ = ch.run(Xo, d.y, G, seed=201 + c, n=n)
        ora.append(bo[burn:])
    mg, smg, vg, svg = pooled(gpu)
    mo, smo, vo, svo = pooled(ora)
    assert np.all(np.abs(mg - mo) <= 4 * np.sqrt(smg**2 + smo**2) + 1e-12)
    assert np.all(np.abs(vg - vo) <= 4 * np.sqrt(svg**2 + svo**2) + 1e-12)
    nz = np.flatnonzero(d.beta_true)
    allg = np.concatenate(gpu)
    lo, hi = np.quantile(allg[:, nz], 0.05, axis=0), np.quantile(allg[:, nz], 0.95, axis=0)
    big = np.abs(d.beta_true[nz]) > 0.5
    assert np.all((np.sign(lo) == np.sign(d.beta_true[nz]))[big])
    assert np.all((np.sign(hi) == np.sign(d.beta_true[nz]))[big])


def check_full_size_z_step(orc, hsp, s, Xo, Xf, y, beta, seed, k):
    """One z step at full size against the oracle, every row."""
    s.step(hsp.HSP_STEP_Z)
    z, att, b = s.debug()
    zo, ao, bo = orc.z_step(Xo, y, beta, seed, k)
    assert np.all(z * (2.0 * y - 1.0) > 0)
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= int(1e-5 * y.size)
    ok = ~flips
    assert np.max(np.abs(z[ok] - zo[ok]) / z_scale(Xf[ok], beta)) < 1e-5
    # X^T z of the kernel's own z, and the oracle's b with the flipped rows' share
    scale = b_scale(Xf, zo)
    assert np.max(np.abs(b - orc.xtz(Xo, z.astype(np.float64))) / b_scale(Xf, z)) < 1e-5
    dz = np.abs(z.astype(np.float64) - zo)
    dz[ok] = 0.0
    slack = np.abs(Xf[flips].astype(np.float64)).T @ dz[flips] if flips.any() else 0.0
    assert np.all(np.abs(b - orc.xtz(Xo, zo)) <= 1e-5 * scale + slack)
    return flips.sum()


def test_full_size_workload(env, orc):
    torch, hsp = env
    d = synth.config3()
    s = hsp.Sampler(d.X, d.y, seed=1, debug_store_z=True, max_draws=64)
    rng = np.random.default_rng(5)
    # G on sampled entries (the oracle sums each entry over all rows)
    G = s.gram()
    for _ in range(24):
        j, k = rng.integers(0, d.p, 2)
        ref = orc.gram_entry(d.X, int(j), int(k))
        assert abs(G[j, k] - ref) <= 1e-12 * math.sqrt(G[j, j] * G[k, k])
    # one z step at a state with realistic |x_i beta|
    beta = np.zeros(d.p)
    beta[d.beta_true != 0] = d.beta_true[d.beta_true != 0]
    beta += rng.normal(0, 0.01, d.p)
    s.set_state(beta, np.ones(d.p), np.ones(d.p), 1.0, 1.0, 30)
    check_full_size_z_step(orc, hsp, s, d.X, d.X, d.y, beta, 1, 31)
    # 50 whole sweeps from the cold start, as timed by the benchmark
    s.set_state(np.zeros(d.p), np.ones(d.p), np.ones(d.p), 1.0, 1.0, 0)
    s.sweep(50)
    z, att, b = s.debug()
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    betas, taus, n = s.draws()
    assert n == 50 and np.all(np.isfinite(betas)) and np.all(taus > 0)
    clamps, maxatt = s.counters()
    assert clamps == 0 and maxatt < 64
    # the chain has moved towards the truth on the nonzero coefficients
    nz = np.flatnonzero(d.beta_true)
    assert np.corrcoef(betas[-1][nz], d.beta_true[nz])[0, 1] > 0.9
    s.close()


def test_full_size_bf16_workload(env, orc):
    """The bfloat16 form at its throughput shape (N = 1e6, p = 1000, 2 GB):
    matched-design parity of the z step and X^T z on every row, G on sampled
    entries, and whole sweeps."""
    torch, hsp = env
    d = synth.config3()
    bits = synth.bf16_bits(d.X).reshape(d.X.shape)
    Xf = synth.bf16_to_f32(bits).reshape(d.X.shape)
    s = hsp.Sampler(d.X, d.y, seed=2, x_type="bf16", debug_store_z=True, max_draws=64)
    rng = np.random.default_rng(6)
    G = s.gram()
    for _ in range(16):
        j, k = rng.integers(0, d.p, 2)
        ref = orc.gram_entry(bits, int(j), int(k))
        assert abs(G[j, k] - ref) <= 1e-12 * math.sqrt(G[j, j] * G[k, k])
    beta = np.zeros(d.p)
    beta[d.beta_true != 0] = d.beta_true[d.beta_true != 0]
    beta += rng.normal(0, 0.01, d.p)
    s.set_state(beta, np.ones(d.p), np.ones(d.p), 1.0, 1.0, 40)
    check_full_size_z_step(orc, hsp, s, bits, Xf, d.y, beta, 2, 41)
    s.set_state(np.zeros(d.p), np.ones(d.p), np.ones(d.p), 1.0, 1.0, 0)
    s.sweep(30)
    z, att, b = s.debug()
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    betas, taus, n = s.draws()
    assert n == 30 and np.all(np.isfinite(betas)) and np.all(taus > 0)
    nz = np.flatnonzero(d.beta_true)
    assert np.corrcoef(betas[-1][nz], d.beta_true[nz])[0, 1] > 0.9
    s.close()
