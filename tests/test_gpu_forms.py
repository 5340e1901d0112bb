"""GPU: the bfloat16-X form, checkpoint/resume, the draw ring, error paths.

The bfloat16 form is held to the float32 bars against the oracle run on the
same bfloat16-rounded design (the "matched design"); against the oracle on the
original float32 X the per-step error is only reported (it is dominated by the
rounding of X itself, ~2^-9 relative per entry).
"""
import numpy as np
import pytest

import synth
from gpu_util import b_scale, dataset, need_gpu, random_state, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


def make(env, d, seed, **kw):
    torch, hsp = env
    return hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=seed, **kw)


# Beyond p = 2048 the bfloat16 z pass holds 4-row tiles.
@pytest.mark.parametrize("N,p", [(5003, 10), (4099, 100), (2051, 257), (2003, 1000), (1501, 2049),
                                 (1000, 4096)])
def test_bf16_matched_design(env, orc, N, p):
    torch, hsp = env
    d = dataset(N, p, 300 + p)
    bits = synth.bf16_bits(d.X).reshape(d.X.shape)
    s = make(env, d, 5, x_type="bf16", debug_store_z=True)
    G = s.gram()
    Gm = orc.gram(bits) if p <= 1000 else orc.gram_fast(bits)
    scale = np.sqrt(np.outer(np.diag(Gm), np.diag(Gm)))
    assert np.max(np.abs(G - Gm) / scale) < 1e-12
    st = random_state(p, 310 + p, beta_scale=1.5 / np.sqrt(p))
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], 9)
    s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    z, att, b = s.debug()
    zo, ao, bo = orc.z_step(bits, d.y, st["beta"], 5, 10)
    Xm = synth.bf16_to_f32(bits).reshape(d.X.shape)
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= int(1e-5 * N)
    assert np.max(np.abs(z - zo) / z_scale(Xm, st["beta"])) < 1e-5
    assert np.max(np.abs(b - orc.xtz(bits, zo)) / b_scale(Xm, zo)) < 1e-5
    # reported, not gated: the same step on the unrounded float32 design
    zf, _, _ = orc.z_step(d.X, d.y, st["beta"], 5, 10)
    rel = np.abs(z - zf) / z_scale(d.X, st["beta"])
    print(f"bf16 vs float32 design: z error median {np.median(rel):.2e}, max {rel.max():.2e}")
    s.close()


def test_checkpoint_resume_is_bit_exact(env):
    torch, hsp = env
    d = dataset(3001, 150, 41)
    a = make(env, d, 77)
    a.sweep(12)
    sa = a.state()
    b = make(env, d, 77)
    b.sweep(6)
    mid = b.state()
    b.close()
    c = make(env, d, 77)
    c.set_state(mid["beta"], mid["lam_m2"], mid["nu_m1"], mid["tau_m2"], mid["xi_m1"], mid["sweep"])
    c.sweep(6)
    sc = c.state()
    for key in ("beta", "lam_m2", "nu_m1"):
        assert np.array_equal(sa[key], sc[key])
    assert sa["tau_m2"] == sc["tau_m2"] and sa["xi_m1"] == sc["xi_m1"] and sc["sweep"] == 12
    a.close()
    c.close()


def test_draw_ring_thin_and_wrap(env):
    torch, hsp = env
    d = dataset(2000, 20, 42)
    s = make(env, d, 3, thin=2, max_draws=5, record_lambda=True)
    s.sweep(14)  # 7 kept draws, ring of 5
    beta, tau, lam, n = s.draws(2, 5)
    assert n == 7
    st = s.state()
    assert np.array_equal(beta[-1], st["beta"]) and tau[-1] == st["tau_m2"]
    assert np.array_equal(lam[-1], st["lam_m2"])
    with pytest.raises(hsp.HspError):
        s.draws(0, 3)  # overwritten
    with pytest.raises(hsp.HspError):
        s.draws(5, 3)  # not recorded yet
    s.close()


def test_same_seed_same_draws_other_seed_differs(env):
    torch, hsp = env
    d = dataset(2500, 30, 43)
    a = make(env, d, 11)
    b = make(env, d, 11)
    c = make(env, d, 12)
    for s in (a, b, c):
        s.sweep(20)
    ba, _, _ = a.draws()
    bb, _, _ = b.draws()
    bc, _, _ = c.draws()
    assert np.array_equal(ba, bb)
    assert not np.array_equal(ba, bc)
    for s in (a, b, c):
        s.close()


def test_not_positive_definite_is_reported_and_poisons(env):
    torch, hsp = env
    d = dataset(1000, 200, 44)
    X = d.X.copy()
    X[:, 7] = 0.0  # a zero column: G has a zero row, Q's pivot 8 is tau * lam_7
    s = hsp.Sampler(torch.from_numpy(X).cuda(), torch.from_numpy(d.y).cuda(), seed=1)
    lam = np.ones(200)
    lam[7] = 0.0
    s.set_state(np.zeros(200), lam, np.ones(200), 1.0, 1.0, 0)
    with pytest.raises(hsp.HspError) as e:
        s.step(hsp.HSP_STEP_Z | hsp.HSP_STEP_BETA)
    assert e.value.code == hsp.HSP_ENOTPD
    with pytest.raises(hsp.HspError) as e:
        s.sweep(1)
    assert e.value.code == hsp.HSP_EPOISONED
    s.close()


def test_invalid_inputs_rejected(env):
    torch, hsp = env
    d = dataset(500, 12, 45)
    y = d.y.copy()
    y[3] = 2
    with pytest.raises(hsp.HspError) as e:
        hsp.Sampler(d.X, y)
    assert e.value.code == hsp.HSP_EINVAL
    X = d.X.copy()
    X[10, 2] = np.nan
    with pytest.raises(hsp.HspError) as e:
        hsp.Sampler(X, d.y)
    assert e.value.code == hsp.HSP_EINVAL
    X = d.X.copy()
    X[10, 2] = np.inf
    with pytest.raises(hsp.HspError) as e:
        hsp.Sampler(X, d.y, x_type="bf16")
    assert e.value.code == hsp.HSP_EINVAL
    # near the float32 limit: bfloat16 rounding would overflow it, but the
    # library stores every column scaled into (-1, 1] first, so it is valid
    X = d.X.copy()
    X[10, 2] = 3.4e38
    s = hsp.Sampler(X, d.y, x_type="bf16")
    G = s.gram()
    big = float(synth.bf16_to_f32(synth.bf16_bits(np.array([3.4e38 * 2.0**-128], np.float32))))
    assert np.isfinite(G).all() and G[2, 2] >= (big * 2.0**128) ** 2
    s.sweep(2)
    assert np.all(np.isfinite(s.state()["beta"]))
    s.close()
    s = hsp.Sampler(d.X, d.y)  # host input path
    with pytest.raises(hsp.HspError) as e:
        s.set_state(np.zeros(12), -np.ones(12), np.ones(12), 1.0, 1.0, 0)
    assert e.value.code == hsp.HSP_EINVAL
    s.sweep(3)
    assert s.state()["sweep"] == 3
    s.close()
