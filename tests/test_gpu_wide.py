"""GPU parity for wide rows (p up to hsp_max_p()), where the z pass splits
every row over the four waves of a block and, beyond p = 4096, the p-side
group takes most of the device (the point (N, p) = (1e6, 1e4) of Sections 6.1
and 7 lies here).  One z step and one beta step from a random state against
the oracle, at the same bars as the narrow rows; G on sampled entries."""
import math

import numpy as np
import pytest

from gpu_util import b_scale, dataset, need_gpu, random_state, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def bits_of(X):
    u = X.view(np.uint32)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


@pytest.mark.parametrize("N,p,xt", [(3001, 4100, "f32"), (1201, 6000, "bf16"), (2003, 4104, "bf16"),
                                    (613, 10000, "f32"), (409, 10240, "f32")])
def test_wide_rows_z_and_beta(env, orc, N, p, xt):
    torch, hsp = env
    d = dataset(N, p, 900 + p % 97)
    Xo = d.X if xt == "f32" else bits_of(d.X)
    Xf = d.X if xt == "f32" else (Xo.astype(np.uint32) << 16).view(np.float32)
    s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=5, x_type=xt,
                    debug_store_z=True)
    G = s.gram()
    rng = np.random.default_rng(p)
    for _ in range(12):
        j, k = rng.integers(0, p, 2)
        ref = orc.gram_entry(Xo, int(j), int(k))
        assert abs(G[j, k] - ref) <= 1e-12 * math.sqrt(G[j, j] * G[k, k])
    st = random_state(p, 910 + p % 89, beta_scale=1.0 / np.sqrt(p))
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], 2)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    z, att, b = s.debug()
    beta_gpu = s.state()["beta"]
    s.close()
    zo, ao, bo = orc.z_step(Xo, d.y, st["beta"], 5, 3)
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= max(1, int(1e-5 * N))
    ok = ~flips
    assert np.max(np.abs(z[ok] - zo[ok]) / z_scale(Xf[ok], st["beta"])) < 1e-5
    assert np.max(np.abs(b - orc.xtz(Xo, z.astype(np.float64))) / b_scale(Xf, z)) < 1e-5
    if p > 10000:
        return  # the float64 oracle's beta step at this size takes minutes
    # beta from the GPU's own z: the oracle's beta step on the same X^T z
    bref = orc.xtz(Xo, z.astype(np.float64))
    Go = orc.gram_fast(Xo)
    beta_o, _, _, rc = orc.beta_step(Go, st["lam_m2"], st["tau_m2"], bref, 5, 3)
    assert rc == 0
    Qi = np.abs(np.linalg.inv(Go + st["tau_m2"] * np.diag(st["lam_m2"])))
    tol = Qi @ (1e-5 * b_scale(Xf, z)) + 1e-10 * np.abs(beta_o)
    assert np.all(np.abs(beta_gpu - beta_o) <= tol), np.max(np.abs(beta_gpu - beta_o) / tol)


def test_wide_rows_sweeps_reproduce(env):
    """Whole sweeps at p = 5000 (float32): graph replay, two runs bit for bit."""
    torch, hsp = env
    d = dataset(20011, 5000, 950)
    out = []
    for _ in range(2):
        s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=8, max_draws=8)
        s.sweep(4)
        betas, taus, n = s.draws()
        out.append((betas, taus))
        assert n == 4 and np.all(np.isfinite(betas)) and np.all(taus > 0)
        s.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
