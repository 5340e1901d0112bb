"""Pins of the oracle's beta step (Section 5, beta steps i-viii).

* Cholesky and both triangular solves against LAPACK (numpy) and scipy.
* The beta conditional against the exact conjugate Gaussian
  N(Q^-1 X^T z, Q^-1), with Q^-1 formed by an explicit inverse -- the
  "naive" formula the paper contrasts with its Cholesky route -- plus the
  chi-square law of the Mahalanobis distance.
* X^T z and X^T X against numpy products of the same float64 values.
"""
import numpy as np
import pytest
import scipy.linalg as sla
from scipy import stats

import synth


def spd(p, seed, cond_boost=0.5):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((p + 5, p))
    return A.T @ A + cond_boost * np.eye(p)


@pytest.mark.parametrize("p", [1, 2, 7, 64, 150])
def test_cholesky_matches_lapack(orc, p):
    Q = spd(p, p)
    U, rc = orc.cholesky_upper(Q)
    assert rc == 0
    L = np.linalg.cholesky(Q)
    np.testing.assert_allclose(U, L.T, rtol=1e-12, atol=1e-12 * np.abs(L).max())
    assert np.all(np.tril(U, -1) == 0.0)


def test_cholesky_reports_non_pd(orc):
    Q = spd(5, 1)
    Q[3, 3] = -1.0
    _, rc = orc.cholesky_upper(Q)
    assert rc == 4
    Q = spd(5, 1)
    Q[0, 0] = np.nan
    _, rc = orc.cholesky_upper(Q)
    assert rc == 1


@pytest.mark.parametrize("p", [1, 5, 80])
def test_triangular_solves_match_scipy(orc, p):
    U = np.triu(spd(p, 10 + p))
    U[np.diag_indices(p)] = np.abs(U.diagonal()) + 1.0
    r = np.random.default_rng(p).standard_normal(p)
    np.testing.assert_allclose(orc.solve_upper(U, r), sla.solve_triangular(U, r, lower=False),
                               rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(orc.solve_upper_t(U, r),
                               sla.solve_triangular(U, r, lower=False, trans="T"),
                               rtol=1e-10, atol=1e-12)


def test_beta_mean_is_explicit_inverse(orc):
    rng = np.random.default_rng(5)
    p = 6
    X = rng.standard_normal((40, p))
    G = X.T @ X
    lam = rng.uniform(0.2, 3.0, p)
    tau = 0.8
    b = rng.standard_normal(p) * 5
    beta, mean, noise, rc = orc.beta_step(G, lam, tau, b, 1, 1)
    assert rc == 0
    Q = G + tau * np.diag(lam)
    np.testing.assert_allclose(mean, np.linalg.inv(Q) @ b, rtol=1e-10)
    np.testing.assert_allclose(beta, mean + noise, rtol=1e-13, atol=1e-15)


def test_beta_draw_law(orc):
    """beta ~ N(Q^-1 b, Q^-1): mean, covariance and Mahalanobis chi-square."""
    rng = np.random.default_rng(6)
    p = 3
    X = rng.standard_normal((12, p))
    G = X.T @ X
    lam = np.array([0.5, 2.0, 9.0])
    tau = 1.7
    b = np.array([3.0, -1.0, 0.5])
    Q = G + tau * np.diag(lam)
    Qi = np.linalg.inv(Q)
    m = Qi @ b
    n = 40_000
    draws = np.array([orc.beta_step(G, lam, tau, b, 99, k)[0] for k in range(1, n + 1)])
    se = np.sqrt(np.diag(Qi) / n)
    assert np.all(np.abs(draws.mean(0) - m) < 5 * se)
    C = np.cov(draws.T)
    assert np.all(np.abs(C - Qi) < 6 * np.sqrt((Qi**2 + np.outer(np.diag(Qi), np.diag(Qi))) / n))
    d = draws - m
    maha = np.einsum("ij,jk,ik->i", d, Q, d)
    assert stats.kstest(maha, stats.chi2(p).cdf).pvalue > 1e-4


def test_xtz_and_gram(orc):
    rng = np.random.default_rng(8)
    X = rng.standard_normal((300, 9)).astype(np.float32)
    z = rng.standard_normal(300)
    X64 = X.astype(np.float64)
    np.testing.assert_allclose(orc.xtz(X, z), X64.T @ z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.gram(X), X64.T @ X64, rtol=1e-12, atol=1e-11)
    assert orc.gram_entry(X, 2, 5) == pytest.approx((X64[:, 2] * X64[:, 5]).sum(), rel=1e-12)
    assert orc.row_dot(X, 17, z[:9]) == pytest.approx(X64[17] @ z[:9], rel=1e-12, abs=1e-12)


def test_bf16_input_is_widened_exactly(orc):
    rng = np.random.default_rng(9)
    X = rng.standard_normal((30, 5)).astype(np.float32)
    bits = synth.bf16_bits(X)
    Xr = synth.bf16_to_f32(bits).reshape(X.shape).astype(np.float64)
    z = rng.standard_normal(30)
    np.testing.assert_allclose(orc.xtz(bits, z), Xr.T @ z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(orc.gram(bits), Xr.T @ Xr, rtol=1e-12, atol=1e-12)
    # bf16 rounding error is at most half an ulp of 8 significant bits
    assert np.all(np.abs(Xr - X) <= np.abs(X) * 2.0**-8 + 1e-30)


def test_gram_fast_is_the_same_sum(orc):
    rng = np.random.default_rng(10)
    X = rng.standard_normal((700, 37)).astype(np.float32)
    X[:, 3] *= 2.0**-20
    X[:, 5] *= 2.0**15
    for Xa in (X, synth.bf16_bits(X).reshape(X.shape)):
        G, Gf = orc.gram(Xa), orc.gram_fast(Xa)
        scale = np.sqrt(np.outer(np.diag(G), np.diag(G)))
        assert np.max(np.abs(G - Gf) / scale) < 1e-13


def test_threads_do_not_change_results(orc):
    """The OpenMP loops keep every sum's order: one thread and many give the
    same bits for the z step, X^T z and the Gram."""
    import synth as _s
    d = _s.probit_design(3000, 70, np.r_[1.0, np.zeros(69)], 5, True)
    beta = np.random.default_rng(1).normal(0, 0.2, 70)
    out = []
    for t in (1, 4):
        orc.set_threads(t)
        z, a, br = orc.z_step(d.X, d.y, beta, 3, 2)
        out.append((z, a, br, orc.xtz(d.X, z), orc.gram(d.X)))
    orc.set_threads(orc.max_threads())
    for u, v in zip(*out):
        assert np.array_equal(u, v)
