"""hsp_gram_noalloc: the Gram of Section 5 (beta step i) through the library's
fixed workspace gives what hsp_gram gives, on consecutive calls that share
that workspace (the second smaller than the first)."""
import numpy as np
import pytest

from gpu_util import need_gpu
import synth

pytestmark = pytest.mark.gpu


def _design(N, p, seed):
    beta, _ = synth.sparse_beta(p, min(5, p - 1), seed, -2.0, 2.0)
    return synth.probit_design(N, p, beta, seed, True, f"n{N}_p{p}").X


def _both(torch, hsp, X, ld, xtype):
    N, p = X.shape
    if xtype == hsp.HSP_X_F32:
        buf = np.zeros((N, ld), np.float32)
        buf[:, :p] = X
    else:
        bits = X.view(np.uint32)
        rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16).astype(np.uint16)
        buf = np.zeros((N, ld), np.uint16)
        buf[:, :p] = rounded
    Xd = torch.from_numpy(buf).cuda()
    G1 = torch.full((p, p), np.nan, dtype=torch.float64, device="cuda")
    G2 = torch.full((p, p), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    hsp.hsp_gram(Xd.data_ptr(), xtype, N, p, ld, G1.data_ptr())
    hsp.hsp_gram_noalloc(Xd.data_ptr(), xtype, N, p, ld, G2.data_ptr())
    Xo = X if xtype == hsp.HSP_X_F32 else np.ascontiguousarray(buf[:, :p])
    return G1.cpu().numpy(), G2.cpu().numpy(), Xo


@pytest.mark.parametrize("xt", ["f32", "bf16"])
def test_gram_noalloc_equals_gram_on_consecutive_calls(orc, xt):
    torch, hsp = need_gpu()
    xtype = hsp.HSP_X_F32 if xt == "f32" else hsp.HSP_X_BF16
    # first call: 136 tile pairs x 8 row splits of 32 KB (34.8 MB) go through
    # the 32 MiB workspace in two rounds; then smaller inputs reuse it
    for (N, p, ld, seed) in [(3001, 1000, 1003, 600), (1501, 130, 136, 601), (777, 10, 10, 602)]:
        X = _design(N, p, seed)
        G1, G2, Xo = _both(torch, hsp, X, ld, xtype)
        assert np.array_equal(G1, G2), (N, p)
        Go = orc.gram(Xo)
        gs = np.sqrt(np.outer(np.diag(Go), np.diag(Go)))
        assert np.max(np.abs(G2 - Go) / gs) < 1e-12, (N, p)


def test_gram_noalloc_rejects_bad_arguments():
    torch, hsp = need_gpu()
    Xd = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    Gd = torch.zeros((8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_gram_noalloc(Xd.data_ptr(), hsp.HSP_X_F32, 10, 8, 4, Gd.data_ptr())
    assert e.value.code == hsp.HSP_EINVAL
    with pytest.raises(hsp.HspError) as e:
        hsp.hsp_gram_noalloc(Xd.data_ptr(), 7, 10, 8, 8, Gd.data_ptr())
    assert e.value.code == hsp.HSP_EINVAL
