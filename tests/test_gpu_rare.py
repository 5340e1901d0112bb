"""GPU: the rare-event workload, a shape-matched stand-in for the data of
Section 6.2 (N = 1,295,848, p = 141, mean outcome 0.0048).

* One z step and one beta step at full size against the oracle (every row;
  X^T z with the flipped rows' share in the bar; beta to the propagated bar).
* A long chain from the cold start: finite draws, the intercept recovered,
  and the truncated-normal branch mix the outcome rate implies (rows with
  y = 0 sit at mu* ~ 3.4 > 0.47, the Gaussian branch; the rare y = 1 rows deep
  in Robert's branch).
"""
import numpy as np
import pytest

import synth
from gpu_util import b_scale, need_gpu, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


@pytest.fixture(scope="module")
def rare():
    return synth.rare_event()


def test_rare_event_one_sweep_parity(env, orc, rare):
    torch, hsp = env
    d = rare
    s = hsp.Sampler(d.X, d.y, seed=5, debug_store_z=True, max_draws=64)
    rng = np.random.default_rng(3)
    beta = d.beta_true + rng.normal(0, 0.01, d.p)
    lam = rng.gamma(2.0, 1.0, d.p)
    s.set_state(beta, lam, np.ones(d.p), 2.0, 1.0, 7)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    z, att, b = s.debug()
    zo, ao, bro = orc.z_step(d.X, d.y, beta, 5, 8)
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bro == 1))
    assert flips.sum() <= int(1e-5 * d.N)
    ok = ~flips
    assert np.max(np.abs(z[ok] - zo[ok]) / z_scale(d.X[ok], beta)) < 1e-5
    dz = np.abs(z.astype(np.float64) - zo)
    dz[ok] = 0.0
    slack = np.abs(d.X[flips].astype(np.float64)).T @ dz[flips] if flips.any() else 0.0
    bo = orc.xtz(d.X, zo)
    assert np.all(np.abs(b - bo) <= 1e-5 * b_scale(d.X, zo) + slack)
    G = orc.gram(d.X)
    beta_o, _, _, rc = orc.beta_step(G, lam, 2.0, bo, 5, 8)
    assert rc == 0
    Qi = np.abs(np.linalg.inv(G + 2.0 * np.diag(lam)))
    tol = Qi @ (1e-5 * b_scale(d.X, zo) + slack) + 1e-10 * np.abs(beta_o)
    assert np.all(np.abs(s.state()["beta"] - beta_o) <= tol)
    s.close()


def test_rare_event_long_chain(env, rare):
    torch, hsp = env
    d = rare
    n, burn = 3000, 750
    s = hsp.Sampler(d.X, d.y, seed=6, debug_store_z=True, max_draws=n)
    s.sweep(n)
    betas, taus, got = s.draws()
    assert got == n and np.all(np.isfinite(betas)) and np.all(taus > 0)
    post = betas[burn:]
    b0 = post[:, 0]
    assert abs(b0.mean() - d.beta_true[0]) < 0.1
    x = b0 - b0.mean()
    rho1 = float(np.dot(x[1:], x[:-1]) / np.dot(x, x))
    print(f"rare-event chain: intercept mean {b0.mean():.4f} (true {d.beta_true[0]:.4f}), "
          f"lag-1 autocorrelation {rho1:.3f}")
    # the branch mix of the last sweep's z step
    z, att, _ = s.debug()
    gauss = (att & (1 << 30)) != 0
    assert np.mean(gauss[d.y == 0]) > 0.99   # mu* = -eta, about 3.4
    assert np.mean(gauss[d.y == 1]) < 0.05   # mu* = eta, about -3.4: Robert's branch
    clamps, maxatt = s.counters()
    assert clamps == 0
    s.close()
