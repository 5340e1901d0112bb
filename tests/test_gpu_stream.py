"""GPU: X streamed from pinned host memory in row chunks (for designs larger
than device memory) draws bit for bit what the same chain draws with X
resident, and one streamed step matches the oracle."""
import numpy as np
import pytest

from gpu_util import b_scale, dataset, need_gpu, random_state, z_scale

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    return need_gpu()


@pytest.mark.parametrize("N,p,xt,rows,on_host", [(200003, 100, "f32", 20000, True),
                                                  (80021, 300, "bf16", 10000, True),
                                                  (50021, 10, "f32", 4096, False),
                                                  (30011, 1000, "f32", 8000, True)])
def test_streamed_chain_equals_resident_chain(env, N, p, xt, rows, on_host):
    torch, hsp = env
    d = dataset(N, p, 800 + p)
    out = []
    for stream in (False, True):
        X = d.X if (stream and on_host) else torch.from_numpy(d.X).cuda()
        y = d.y if (stream and on_host) else torch.from_numpy(d.y).cuda()
        s = hsp.Sampler(X, y, seed=17, x_type=xt, x_stream=stream, stream_rows=rows, max_draws=64,
                        debug_store_z=True, record_lambda=True)
        if stream:
            assert s.plan()[4].startswith("streamed")
        G = s.gram()
        s.sweep(12)
        betas, taus, lams, _ = s.draws()
        z, att, b = s.debug()
        out.append((G, betas, taus, lams, z, att, b))
        s.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_streamed_step_matches_oracle(env, orc):
    torch, hsp = env
    N, p = 70001, 130
    d = dataset(N, p, 831)
    s = hsp.Sampler(d.X, d.y, seed=9, x_stream=True, stream_rows=8000, debug_store_z=True)
    st = random_state(p, 832, beta_scale=1.0 / np.sqrt(p))
    s.set_state(st["beta"], st["lam_m2"], st["nu_m1"], st["tau_m2"], st["xi_m1"], 3)
    s.step(hsp.HSP_STEP_Z)
    z, att, b = s.debug()
    zo, ao, bo = orc.z_step(d.X, d.y, st["beta"], 9, 4)
    assert np.all(z * (2.0 * d.y - 1.0) > 0)
    flips = ((att & ~(1 << 30)) != ao) | (((att & (1 << 30)) != 0) != (bo == 1))
    assert flips.sum() <= int(1e-5 * N)
    ok = ~flips
    assert np.max(np.abs(z[ok] - zo[ok]) / z_scale(d.X[ok], st["beta"])) < 1e-5
    assert np.max(np.abs(b - orc.xtz(d.X, z.astype(np.float64))) / b_scale(d.X, z)) < 1e-5
    # timing and the link ceiling work on a streamed state
    s.set_timing(True)
    s.sweep(3)
    s.sync()
    k_ms, sweep_ms, n = s.timing()
    assert n == 3 and k_ms > 0
    ms, nbytes = hsp.hsp_read_ceiling(s.h, 2)
    assert ms > 0 and nbytes == N * ((p + 3) // 4 * 4) * 4
    s.close()
