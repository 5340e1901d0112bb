"""GPU parity: every conditional of the HIP library against the FP64 oracle.

Both sides receive the same inputs and the same Philox counters, so single
steps are compared element by element.  Tolerances (float32 N-side work):
  z     |dz| <= 1e-5 * max(|z|, sum_j |x_ij beta_j|, 1)
  b     |db_j| <= 1e-5 * sum_i |x_ij z_i|
  beta  |dbeta| <= |Q^-1| (1e-5 * sum_i |x_ij z_i|)  (a 1e-5 relative change of b)
        + 1e-10 |beta|
p-side conditionals fed identical float64 state agree to 1e-12 relative.
Rows whose accepted proposal or branch differs (a float32 vs float64
decision right at a threshold) are counted and must be at most 1e-5 of the
rows; the sign invariant z_i > 0 <=> y_i = 1 must hold exactly.
"""
import numpy as np
import pytest

from gpu_util import b_scale, dataset, need_gpu, random_state, z_scale

pytestmark = pytest.mark.gpu

# p = 16 is the largest p of the one-block p-side path, p = 17 the smallest of
# the tiled one (a single 64-wide tile).  Beyond p = 1024 (float32) the z pass
# holds 4-row tiles, beyond p = 1792 2-row tiles; p = 4096 is the largest p
# (64 x 64 tiles of the factorisation).
SHAPES = [(5003, 2), (5003, 10), (4001, 16), (4001, 17), (4099, 100), (3001, 130), (2051, 257),
          (2003, 1000), (2003, 1025), (1501, 2049), (1000, 4096)]


def gram_of(orc, X):
    """The oracle's G; for large p the same definition by a library matmul."""
    return orc.gram(X) if X.shape[1] <= 1000 else orc.gram_fast(X)


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def make(env, d, seed, **kw):
    torch, hsp = env
    X = torch.from_numpy(d.X).cuda()
    y = torch.from_numpy(d.y).cuda()
    return hsp.Sampler(X, y, seed=seed, debug_store_z=True, **kw)


def test_philox_bit_exact(env, orc):
    torch, hsp = env
    rng = np.random.default_rng(4)
    ctr = rng.integers(0, 2**32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0xDEADBEEF12345678
    out = hsp.hsp_philox(seed, ctr)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint32)
    ref = np.array([orc.philox(c, key) for c in ctr])
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("N,p", SHAPES)
def test_gram(env, orc, N, p):
    d = dataset(N, p, 10 + p)
    s = make(env, d, 1)
    G = s.gram()
    Go = gram_of(orc, d.X)
    scale = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
    assert np.max(np.abs(G - Go) / scale) < 1e-12
    assert np.array_equal(G, G.T)
    s.close()


@pytest.mark.parametrize("N,p", SHAPES)
def test_z_step(env, orc, N, p):
    torch, hsp = env
    d = dataset(N, p, 20 + p)
    s = make(env, d, 7, chain_id=3)
    st = random_state(p, 30 + p, beta_scale=1.5 / np.sqrt(p))
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], 41)
    s.step(hsp.HSP_STEP_Z)
    z, att, b = s.debug()
    zo, ao, bo = orc.z_step(d.X, d.y, st["beta"], 7, 42, chain=3)
    ys = 2.0 * d.y - 1.0
    assert np.all(z * ys > 0), "sign invariant"
    gauss = (att & (1 << 30)) != 0
    flips = ((att & ~(1 << 30)) != ao) | (gauss != (bo == 1))
    assert flips.sum() <= int(1e-5 * N), f"{flips.sum()} rows took another proposal or branch"
    err = np.abs(z - zo) / z_scale(d.X, st["beta"])
    assert err.max() < 1e-5, err.max()
    e_b = np.abs(b - orc.xtz(d.X, zo)) / b_scale(d.X, zo)
    assert e_b.max() < 1e-5, e_b.max()
    # both branches occur at these scales
    assert 0 < gauss.sum() < N
    s.close()


@pytest.mark.parametrize("N,p", [(5003, 10), (2003, 300)])
def test_hyper_steps(env, orc, N, p):
    torch, hsp = env
    d = dataset(N, p, 50 + p)
    s = make(env, d, 11, chain_id=1)
    st = random_state(p, 60 + p)
    k0 = 17
    # lambda alone
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], k0)
    s.step(hsp.HSP_STEP_LAMBDA)
    g = s.state()
    lam_o, _ = orc.lambda_step(st["beta"], st["nu_m1"], st["tau_m2"], 11, k0 + 1, chain=1)
    np.testing.assert_allclose(g["lam_m2"], lam_o, rtol=1e-12)
    # tau alone (uses the state's lambda)
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], k0)
    s.step(hsp.HSP_STEP_TAU)
    tau_o, _ = orc.tau_step(st["lam_m2"], st["beta"], st["xi_m1"], 11, k0 + 1, chain=1)
    assert s.state()["tau_m2"] == pytest.approx(tau_o, rel=1e-12)
    # nu and xi
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], k0)
    s.step(hsp.HSP_STEP_NUXI)
    g = s.state()
    np.testing.assert_allclose(g["nu_m1"], orc.nu_step(st["lam_m2"], 11, k0 + 1, chain=1), rtol=1e-12)
    assert g["xi_m1"] == pytest.approx(orc.xi_step(st["tau_m2"], 11, k0 + 1, chain=1), rel=1e-12)
    s.close()


def beta_tol(G, lam, tau, X, z, beta):
    Q = G + tau * np.diag(lam)
    Qi = np.abs(np.linalg.inv(Q))
    return Qi @ (1e-5 * b_scale(X, z)) + 1e-10 * np.abs(beta)


@pytest.mark.parametrize("N,p", SHAPES)
def test_beta_step(env, orc, N, p):
    torch, hsp = env
    d = dataset(N, p, 70 + p)
    s = make(env, d, 13)
    st = random_state(p, 80 + p, beta_scale=1.0 / np.sqrt(p))
    k0 = 5
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], k0)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    beta_gpu = s.state()["beta"]
    G = gram_of(orc, d.X)
    zo, _, _ = orc.z_step(d.X, d.y, st["beta"], 13, k0 + 1)
    bo = orc.xtz(d.X, zo)
    beta_o, mean_o, noise_o, rc = orc.beta_step(G, st["lam_m2"], st["tau_m2"], bo, 13, k0 + 1)
    assert rc == 0
    tol = beta_tol(G, st["lam_m2"], st["tau_m2"], d.X, zo, beta_o)
    assert np.all(np.abs(beta_gpu - beta_o) <= tol), np.max(np.abs(beta_gpu - beta_o) / tol)
    s.close()


@pytest.mark.parametrize("N,p", [(5003, 10), (4001, 17), (4099, 100), (2051, 257)])
def test_sweep_trajectory(env, orc, N, p):
    """Five whole sweeps from the cold start, state compared after each."""
    torch, hsp = env
    d = dataset(N, p, 90 + p)
    s = make(env, d, 21)
    G = orc.gram(d.X)
    ch = orc.Chain(p)
    allsteps = (hsp.HSP_STEP_Z | hsp.HSP_STEP_LAMBDA | hsp.HSP_STEP_TAU | hsp.HSP_STEP_BETA
                | hsp.HSP_STEP_NUXI | hsp.HSP_STEP_ADVANCE)
    for k in range(1, 6):
        beta_prev = ch.beta.copy()
        s.step(allsteps)
        z, att, b = s.debug()
        zo, bo, _ = ch.sweep_once(d.X, d.y, G, seed=21, want_z=True)
        assert np.all(z * (2.0 * d.y - 1.0) > 0)
        assert np.max(np.abs(z - zo) / z_scale(d.X, beta_prev)) < 1e-5
        g = s.state()
        assert g["sweep"] == ch.sweep == k
        tol = beta_tol(G, ch.lam_m2, ch.tau_m2, d.X, zo, ch.beta) * 10
        assert np.all(np.abs(g["beta"] - ch.beta) <= tol)
        for key, ref in [("lam_m2", ch.lam_m2), ("nu_m1", ch.nu_m1)]:
            np.testing.assert_allclose(g[key], ref, rtol=1e-4)
        assert g["tau_m2"] == pytest.approx(ch.tau_m2, rel=1e-4)
        assert g["xi_m1"] == pytest.approx(ch.xi_m1, rel=1e-4)
    s.close()


def test_graph_sweeps_equal_steps_and_reproduce(env):
    """hsp_sweep (graph replay) equals step-by-step sweeps bit for bit, run to run."""
    torch, hsp = env
    d = dataset(3001, 40, 5)
    allsteps = (hsp.HSP_STEP_Z | hsp.HSP_STEP_LAMBDA | hsp.HSP_STEP_TAU | hsp.HSP_STEP_BETA
                | hsp.HSP_STEP_NUXI | hsp.HSP_STEP_ADVANCE)
    a = make(env, d, 99)
    a.sweep(7)
    sa = a.state()
    beta_a, tau_a, n = a.draws()
    assert n == 7
    b = make(env, d, 99)
    for _ in range(7):
        b.step(allsteps)
    sb = b.state()
    c = make(env, d, 99, use_graph=False)
    c.sweep(7)
    sc = c.state()
    for key in ("beta", "lam_m2", "nu_m1"):
        assert np.array_equal(sa[key], sb[key]) and np.array_equal(sa[key], sc[key])
    assert sa["tau_m2"] == sb["tau_m2"] == sc["tau_m2"]
    assert np.array_equal(beta_a[-1], sa["beta"]) and tau_a[-1] == sa["tau_m2"]
    for s in (a, b, c):
        s.close()
