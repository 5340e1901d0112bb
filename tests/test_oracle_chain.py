"""Whole-chain pins of the oracle sampler.

* X = 0: the likelihood carries no information, so the chain must sample the
  horseshoe prior of Eq. (10): lambda_j and tau half-Cauchy C+(0,1)
  (quartiles tan(pi/8), 1, tan(3 pi/8)), and beta_j / (lambda_j tau) ~ N(0,1).
* p = 2 with lambda, tau frozen: the (z, beta) chain targets
  prod_i Phi(y*_i x_i beta) N(beta; 0, tau^2 Lambda^2), whose mean and
  variance are computed exactly on a fine 2-D grid.
* Recovery (Section 6.1): the posterior identifies the nonzero coefficients
  and shrinks the zero ones.
"""
import math

import numpy as np
import pytest
from scipy import stats

import synth


def batch_means_se(x, nb=None):
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    nb = nb or int(math.sqrt(n))
    m = n // nb
    bm = x[: nb * m].reshape(nb, m, *x.shape[1:]).mean(1)
    return bm.std(0, ddof=1) / math.sqrt(nb)


def test_zero_design_samples_the_prior(orc):
    p, N = 4, 2
    X = np.zeros((N, p), np.float32)
    y = np.array([1, 0], np.uint8)
    c = orc.Chain(p)
    beta, tau, lam = c.run(X, y, np.zeros((p, p)), seed=5, n=300_000, record_lambda=True)
    burn = 2000
    lam_s = 1.0 / np.sqrt(lam[burn:])
    tau_s = 1.0 / np.sqrt(tau[burn:])
    for q, prob in [(math.tan(math.pi / 8), 0.25), (1.0, 0.5), (math.tan(3 * math.pi / 8), 0.75)]:
        ind_l = (lam_s < q).astype(float)
        ind_t = (tau_s < q).astype(float)
        assert np.all(np.abs(ind_l.mean(0) - prob) < 5 * batch_means_se(ind_l) + 1e-3)
        assert abs(ind_t.mean() - prob) < 5 * batch_means_se(ind_t) + 1e-3
    # beta_j given the same sweep's lambda_j, tau is exactly N(0, lambda_j^2 tau^2)
    std = beta[burn:] * np.sqrt(lam[burn:] * tau[burn:, None])
    assert stats.kstest(std.ravel()[::7], stats.norm.cdf).pvalue > 1e-4


def grid_posterior(X, y, prior_var, half_width=6.0, n=401):
    """Exact mean/variance of prod Phi(y* x beta) N(beta; 0, diag(prior_var)) on a grid."""
    ys = 2.0 * y - 1.0
    # centre the grid with a few Newton-free moment passes on a coarse grid
    c = np.zeros(2)
    s = np.sqrt(prior_var)
    for _ in range(2):
        g0 = np.linspace(c[0] - half_width * s[0], c[0] + half_width * s[0], n)
        g1 = np.linspace(c[1] - half_width * s[1], c[1] + half_width * s[1], n)
        B0, B1 = np.meshgrid(g0, g1, indexing="ij")
        eta = X[:, 0, None, None] * B0 + X[:, 1, None, None] * B1
        logw = stats.norm.logcdf(ys[:, None, None] * eta).sum(0)
        logw += -0.5 * (B0**2 / prior_var[0] + B1**2 / prior_var[1])
        w = np.exp(logw - logw.max())
        w /= w.sum()
        m = np.array([(w * B0).sum(), (w * B1).sum()])
        v = np.array([(w * (B0 - m[0]) ** 2).sum(), (w * (B1 - m[1]) ** 2).sum()])
        c, s = m, np.sqrt(v)
    return m, v


def test_p2_grid_posterior(orc):
    rng = np.random.default_rng(21)
    N, p = 50, 2
    X = rng.standard_normal((N, p)).astype(np.float32)
    y = (X.astype(np.float64) @ np.array([1.0, -0.5]) + rng.standard_normal(N) > 0).astype(np.uint8)
    lam_m2 = np.array([0.8, 2.5])
    tau_m2 = 1.3
    prior_var = 1.0 / (tau_m2 * lam_m2)
    m_exact, v_exact = grid_posterior(X.astype(np.float64), y, prior_var)

    G = orc.gram(X)
    beta = np.zeros(p)
    n, burn = 40_000, 500
    draws = np.empty((n, p))
    for k in range(1, n + burn + 1):
        z, _, _ = orc.z_step(X, y, beta, 31, k)
        b = orc.xtz(X, z)
        beta, _, _, rc = orc.beta_step(G, lam_m2, tau_m2, b, 31, k)
        assert rc == 0
        if k > burn:
            draws[k - burn - 1] = beta
    se_m = batch_means_se(draws)
    assert np.all(np.abs(draws.mean(0) - m_exact) < 4 * se_m + 1e-3)
    sq = (draws - m_exact) ** 2
    assert np.all(np.abs(sq.mean(0) - v_exact) < 4 * batch_means_se(sq) + 1e-3)


def test_recovery_small_design(orc):
    """Section 6.1: nonzero coefficients identified, zero ones shrunk."""
    d = synth.config1()
    G = orc.gram(d.X)
    c = orc.Chain(d.p)
    beta, tau = c.run(d.X, d.y, G, seed=1, n=3000)
    post = beta[750:]
    lo, hi = np.quantile(post, 0.05, axis=0), np.quantile(post, 0.95, axis=0)
    for j in np.flatnonzero(d.beta_true):
        assert np.sign(lo[j]) == np.sign(hi[j]) == np.sign(d.beta_true[j])
    zero = d.beta_true == 0
    assert np.median(np.abs(np.median(post[:, zero], axis=0))) < 0.15
    assert np.all(np.isfinite(tau))
