"""GPU: reordering the stored rows by y* x_i beta (Section 5's suggestion for
after burn-in) keeps every row's truncated-normal draw bit for bit, keeps
X^T z within the float32 bar, and the chain keeps matching the oracle."""
import numpy as np
import pytest

import synth
from gpu_util import b_scale, dataset, need_gpu, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


@pytest.mark.parametrize("N,p,xt", [(100003, 100, "f32"), (60013, 300, "bf16"), (30011, 2000, "f32")])
def test_sorted_rows_draw_the_same_z(env, orc, N, p, xt):
    torch, hsp = env
    d = dataset(N, p, 1000 + p)
    mk = lambda: hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=12,
                             x_type=xt, debug_store_z=True, max_draws=64)
    a, b = mk(), mk()
    a.sweep(15)  # burn-in
    st = a.state()
    b.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], st["sweep"])
    a.sort_rows()
    G0 = b.gram()
    assert np.array_equal(a.gram(), G0)
    for s in (a, b):
        s.step(hsp.HSP_STEP_Z)
    za, aa, ba = a.debug()
    zb, ab, bb = b.debug()
    assert np.array_equal(za, zb) and np.array_equal(aa, ab)
    if xt == "f32":
        Xo, Xf = d.X, d.X
    else:
        Xo = synth.bf16_bits(d.X).reshape(d.X.shape)
        Xf = synth.bf16_to_f32(Xo).reshape(d.X.shape)
    scale = b_scale(Xf, za)
    assert np.max(np.abs(ba - bb) / scale) < 1e-5
    # against the oracle on the matched design
    zo, ao, bo = orc.z_step(Xo, d.y, st["beta"], 12, st["sweep"] + 1)
    flips = ((aa & ~(1 << 30)) != ao) | (((aa & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= max(1, int(1e-5 * N))
    ok = ~flips
    assert np.max(np.abs(za[ok] - zo[ok]) / z_scale(Xf[ok], st["beta"])) < 1e-5
    assert np.max(np.abs(ba - orc.xtz(Xo, za.astype(np.float64))) / scale) < 1e-5
    # the sorted chain sweeps on: finite draws, the sign invariant, reproducible
    a.sweep(10)
    betas, taus, _ = a.draws()
    z, _, _ = a.debug()
    assert np.all(np.isfinite(betas)) and np.all(taus > 0)
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    a.close()
    b.close()


def test_sorting_twice_and_rejections(env):
    torch, hsp = env
    d = dataset(20011, 40, 1101)
    s = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=3, debug_store_z=True)
    s.sweep(5)
    s.sort_rows()
    s.sweep(3)
    s.sort_rows()  # composes with the first order
    st = s.state()
    r = hsp.Sampler(torch.from_numpy(d.X).cuda(), torch.from_numpy(d.y).cuda(), seed=3, debug_store_z=True)
    r.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], st["sweep"])
    s.step(hsp.HSP_STEP_Z)
    r.step(hsp.HSP_STEP_Z)
    assert np.array_equal(s.debug()[0], r.debug()[0])
    s.close()
    r.close()
    st2 = hsp.Sampler(d.X, d.y, seed=3, x_stream=True, stream_rows=4096)
    with pytest.raises(hsp.HspError) as e:
        st2.sort_rows()
    assert e.value.code == hsp.HSP_EINVAL
    st2.close()
