"""GPU parity on designs whose columns live on very different scales, on a
nearly collinear design, and of the stand-alone Gram entry point.

The library stores every column of X multiplied by the power of two that
brings its largest magnitude into (1/2, 1], so the grid on which X^T z is
accumulated follows each column's scale.  These tests hold z, b = X^T z and
beta to the same bars as the iid N(0,1) designs when columns are scaled by
2^-30 ... 2^28 (and by scales that are not powers of two), including a
column whose |b_j| exceeds 2^29, for float32 and bfloat16 storage.
"""
import numpy as np
import pytest

import synth
from gpu_util import b_scale, dataset, need_gpu, random_state, z_scale

pytestmark = pytest.mark.gpu

SCALES = [1.0, 2.0**-30, 2.0**-10, 2.0**12, 3.0 * 2.0**-20, 0.7 * 2.0**7, 2.0**28, 1.0]


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def scaled_design(N, p, seed):
    d = dataset(N, p, seed)
    s = np.array([SCALES[j % len(SCALES)] for j in range(p)])
    s[0] = 1.0  # the intercept column stays 1
    X = (d.X.astype(np.float64) * s).astype(np.float32)
    return X, d.y, s


def matched(X, xt):
    """(oracle input, its float32 values) for the storage type."""
    if xt == "bf16":
        bits = synth.bf16_bits(X).reshape(X.shape)
        return bits, synth.bf16_to_f32(bits).reshape(X.shape)
    return X, X


def beta_tol(G, lam, tau, Xf, z, beta):
    Qi = np.abs(np.linalg.inv(G + tau * np.diag(lam)))
    return Qi @ (1e-5 * b_scale(Xf, z)) + 1e-10 * np.abs(beta)


@pytest.mark.parametrize("xt", ["f32", "bf16"])
@pytest.mark.parametrize("N,p", [(5003, 16), (4099, 40), (2051, 257)])
def test_scaled_columns_z_b_beta(env, orc, xt, N, p):
    torch, hsp = env
    X, y, scale = scaled_design(N, p, 500 + p)
    Xo, Xf = matched(X, xt)
    s = hsp.Sampler(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), seed=7, x_type=xt,
                    debug_store_z=True)
    G = s.gram()
    Go = orc.gram(Xo)
    gs = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
    assert np.max(np.abs(G - Go) / gs) < 1e-12
    st = random_state(p, 510 + p, beta_scale=1.5 / np.sqrt(p))
    beta = st["beta"] / scale  # x_ij beta_j of the usual size in every column
    s.set_state(beta, st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], 12)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    z, att, b = s.debug()
    zo, ao, bo = orc.z_step(Xo, y, beta, 7, 13)
    assert np.all(z * (2.0 * y - 1.0) > 0), "sign invariant"
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= int(1e-5 * N)
    assert np.max(np.abs(z - zo) / z_scale(Xf, beta)) < 1e-5
    bref = orc.xtz(Xo, zo)
    assert np.max(np.abs(b - bref) / b_scale(Xf, zo)) < 1e-5
    assert np.max(np.abs(bref)) > 2.0**29  # the 2^28 columns
    beta_o, _, _, rc = orc.beta_step(Go, st["lam_m2"], st["tau_m2"], bref, 7, 13)
    assert rc == 0
    tol = beta_tol(Go, st["lam_m2"], st["tau_m2"], Xf, zo, beta_o)
    assert np.all(np.abs(s.state()["beta"] - beta_o) <= tol)
    s.close()


@pytest.mark.parametrize("xt", ["f32", "bf16"])
def test_scaled_columns_reproducible_and_whole_sweeps(env, orc, xt):
    """Three whole sweeps; two runs agree bit for bit, and every sweep matches
    one oracle sweep from the GPU's own state before it (the single-sweep
    bars).  Coefficients of the 2^-30 columns are set by the prior, so tau^-2
    carries the other coefficients' X^T z rounding into them from one sweep to
    the next (Eq. 12): a trajectory is compared sweep by sweep, not end to end."""
    torch, hsp = env
    X, y, scale = scaled_design(6007, 24, 520)
    Xo, Xf = matched(X, xt)
    runs = []
    for _ in range(2):
        s = hsp.Sampler(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), seed=3, x_type=xt,
                        debug_store_z=True, record_lambda=True)
        s.sweep(3)
        runs.append((s.draws(), s.debug()[2]))
        s.close()
    (b1, t1, l1, _), bb1 = runs[0]
    (b2, t2, l2, _), bb2 = runs[1]
    assert np.array_equal(b1, b2) and np.array_equal(t1, t2) and np.array_equal(l1, l2)
    assert np.array_equal(bb1, bb2)
    G = orc.gram(Xo)
    for k in range(1, 4):
        if k == 1:
            ch = orc.Chain(24)  # the cold start
        else:
            # the state after sweep k - 1: nu and xi are that sweep's draws from its
            # lambda and tau (the same counters on both sides)
            lam, tau = l1[k - 2], t1[k - 2]
            ch = orc.Chain(24, beta=b1[k - 2], lam_m2=lam, nu_m1=orc.nu_step(lam, 3, k - 1),
                           tau_m2=tau, xi_m1=orc.xi_step(tau, 3, k - 1), sweep=k - 1)
        zo, bo, _ = ch.sweep_once(Xo, y, G, seed=3, want_z=True)
        tol = beta_tol(G, ch.lam_m2, ch.tau_m2, Xf, zo, ch.beta)
        assert np.all(np.abs(b1[k - 1] - ch.beta) <= tol), k
        np.testing.assert_allclose(l1[k - 1], ch.lam_m2, rtol=1e-12)
        assert t1[k - 1] == pytest.approx(ch.tau_m2, rel=1e-12)
    assert np.max(np.abs(bb1 - bo) / b_scale(Xf, zo)) < 1e-5


@pytest.mark.parametrize("xt", ["f32", "bf16"])
def test_hsp_gram_matches_oracle_and_sampler(env, orc, xt):
    """hsp_gram on a strided device matrix; the same G, bit for bit, as the
    sampler forms from its column-scaled copy (power-of-two scaling is exact)."""
    torch, hsp = env
    X, y, _ = scaled_design(3001, 70, 530)
    Xo, _ = matched(X, xt)
    ld = 77
    if xt == "f32":
        buf = np.zeros((X.shape[0], ld), np.float32)
        buf[:, :70] = X
        xtype = hsp.HSP_X_F32
    else:
        buf = np.zeros((X.shape[0], ld), np.uint16)
        buf[:, :70] = Xo
        xtype = hsp.HSP_X_BF16
    Xd = torch.from_numpy(buf).cuda()
    Gd = torch.zeros((70, 70), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    hsp.hsp_gram(Xd.data_ptr(), xtype, X.shape[0], 70, ld, Gd.data_ptr())
    G = Gd.cpu().numpy()
    Go = orc.gram(Xo)
    gs = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
    assert np.max(np.abs(G - Go) / gs) < 1e-12
    assert np.array_equal(G, G.T)
    s = hsp.Sampler(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), x_type=xt)
    assert np.array_equal(s.gram(), G)
    s.close()
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_gram(Xd.data_ptr(), xtype, X.shape[0], 70, 60, Gd.data_ptr())
    assert e.value.code == hsp.HSP_EINVAL


def test_near_collinear_columns(env, orc):
    """Two columns with correlation 1 - 1e-8: beta through the explicit L^-1
    agrees with the oracle's substitutions within the bound the conditioning
    of Q allows."""
    torch, hsp = env
    N, p = 5003, 60
    d = dataset(N, p, 540)
    rng = np.random.default_rng(541)
    X = d.X.copy()
    eps = np.sqrt(2e-8)
    X[:, 2] = (X[:, 1].astype(np.float64) + eps * rng.standard_normal(N)).astype(np.float32)
    corr = np.corrcoef(X[:, 1].astype(np.float64), X[:, 2].astype(np.float64))[0, 1]
    assert 1 - 3e-8 < corr < 1 - 3e-9
    s = hsp.Sampler(torch.from_numpy(X).cuda(), torch.from_numpy(d.y).cuda(), seed=9, debug_store_z=True)
    st = random_state(p, 542, beta_scale=1.0 / np.sqrt(p))
    lam = np.full(p, 1e-3)
    tau = 1.0
    s.set_state(st["beta"], lam, st["nu_m1"], tau, st["xi_m1"], 4)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    beta_gpu = s.state()["beta"]
    G = orc.gram(X)
    Q = G + tau * np.diag(lam)
    cond = np.linalg.cond(Q)
    assert cond > 1e6
    zo, _, _ = orc.z_step(X, d.y, st["beta"], 9, 5)
    bo = orc.xtz(X, zo)
    beta_o, _, _, rc = orc.beta_step(G, lam, tau, bo, 9, 5)
    assert rc == 0
    tol = beta_tol(G, lam, tau, X, zo, beta_o) + 64 * 2.0**-52 * cond * np.max(np.abs(beta_o))
    assert np.all(np.abs(beta_gpu - beta_o) <= tol), np.max(np.abs(beta_gpu - beta_o) / tol)
    s.close()
