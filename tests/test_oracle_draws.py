"""Pins of the oracle's single-variable draws against closed forms.

* Truncated normal (Section 5, z step ii): moments of N(mu, 1) truncated to
  the half-line, a KS test against scipy's truncnorm, the acceptance rate of
  each branch against its closed form, the exact sign invariant, and the
  paper's 0.47 threshold / "around 2/3" worst-case acceptance.
* Cheng's gamma (Section 5, tau^-2 step iii): moments, KS against scipy's
  gamma law, and the per-proposal acceptance 1/M of algorithm GB against its
  closed form (and the paper's "approximately 0.88").
* Exponential draws by inversion (Section 5, lambda / nu / xi steps): KS
  against the exponential law with the rate of Eq. (12).
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import special, stats

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def tn_batch(orc, mu_star, y, n, seed=7, sweep=1):
    """n draws of TN(eta, 1, y) with y* eta = mu_star, one row each."""
    X = np.ones((n, 1), np.float32)
    ys = 1.0 if y else -1.0
    beta = np.array([ys * mu_star])
    z, att, br = orc.z_step(X, np.full(n, y, np.uint8), beta, seed, sweep)
    return z, att, br


def tn_moments(mu):
    """Mean and variance of N(mu, 1) truncated to (0, inf)."""
    lam = stats.norm.pdf(mu) / stats.norm.cdf(mu)
    return mu + lam, 1.0 - mu * lam - lam * lam


def robert_acceptance(mu):
    theta = (-mu + math.sqrt(mu * mu + 4.0)) / 2.0
    return theta * math.sqrt(2 * math.pi) * math.exp(-theta * mu - theta * theta / 2) * stats.norm.cdf(mu)


MUS = [-6.0, -2.0, -0.5, 0.0, 0.3, 0.47, 0.471, 0.9, 2.0, 5.0]


@pytest.mark.parametrize("mu", MUS)
@pytest.mark.parametrize("y", [0, 1])
def test_tn_moments_ks_sign(orc, mu, y):
    n = 40_000
    z, att, br = tn_batch(orc, mu, y, n, seed=100 + int(10 * mu) + y)
    ys = 1.0 if y else -1.0
    # exact sign invariant: z > 0 iff y = 1
    assert np.all(ys * z > 0.0)
    assert np.all(att >= 0)
    t = ys * z  # t ~ N(mu, 1) restricted to (0, inf)
    m, v = tn_moments(mu)
    assert abs(t.mean() - m) < 5 * math.sqrt(v / n)
    # variance of the sample variance ~ (mu4 - v^2)/n; use a loose 6-sigma bound
    assert abs(t.var() - v) < 6 * v * math.sqrt(3.0 / n)
    a = -mu  # lower bound of the standardised variable
    ks = stats.kstest(t, stats.truncnorm(a, np.inf, loc=mu, scale=1.0).cdf)
    assert ks.pvalue > 1e-4
    # branch choice follows the 0.47 threshold of Section 5
    expect_gauss = np.float32(mu) > np.float32(GOLD["tn_branch_threshold"]["value"])
    assert np.all(br == (1 if expect_gauss else 0))


@pytest.mark.parametrize("mu", MUS)
def test_tn_acceptance_rates(orc, mu):
    n = 60_000
    z, att, br = tn_batch(orc, mu, 1, n, seed=900 + int(100 * mu))
    first = np.mean(att == 0)
    pred = stats.norm.cdf(mu) if br[0] == 1 else robert_acceptance(mu)
    assert abs(first - pred) < 5 * math.sqrt(pred * (1 - pred) / n) + 1e-12
    # the number of attempts is geometric with that success probability
    assert abs(np.mean(att + 1) - 1.0 / pred) < 6 * math.sqrt((1 - pred) / pred**2 / n)


def test_tn_threshold_is_equal_acceptance_crossover():
    """0.47 is where both samplers accept equally often, at about 2/3 (Section 5)."""
    thr = GOLD["tn_branch_threshold"]["value"]
    f = lambda m: stats.norm.cdf(m) - robert_acceptance(m)
    from scipy.optimize import brentq
    cross = brentq(f, 0.0, 1.0)
    assert abs(cross - thr) < 5e-3
    worst = stats.norm.cdf(thr)
    assert abs(worst - GOLD["tn_worst_case_acceptance"]["value"]) < 0.02


def test_tn_worst_case_acceptance_of_oracle(orc):
    """The oracle's empirical acceptance is lowest next to 0.47, at about 2/3."""
    grid = [-2.0, -1.0, 0.0, 0.3, 0.44, 0.47, 0.5, 0.8, 1.5]
    acc = []
    for m in grid:
        _, att, _ = tn_batch(orc, m, 1, 30_000, seed=3000 + int(100 * m))
        acc.append(np.mean(att == 0))
    acc = np.array(acc)
    i = int(np.argmin(acc))
    assert grid[i] in (0.44, 0.47, 0.5)
    assert abs(acc[i] - 2.0 / 3.0) < 0.03
    assert np.all(acc > 0.66)


def test_tn_half_normal_at_zero(orc):
    """At beta = 0 every z_i is y* |N(0,1)|: mean +-sqrt(2/pi), variance 1 - 2/pi."""
    n = 50_000
    for y in (0, 1):
        z, _, _ = tn_batch(orc, 0.0, y, n, seed=55 + y)
        ys = 1.0 if y else -1.0
        assert abs(z.mean() - ys * math.sqrt(2 / math.pi)) < 5 * math.sqrt((1 - 2 / math.pi) / n)
        assert abs(z.var() - (1 - 2 / math.pi)) < 0.02


def test_tn_draw_matches_z_step(orc):
    """Single-row entry point and the row loop draw the same numbers."""
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, 4)).astype(np.float32)
    y = (rng.random(50) < 0.5).astype(np.uint8)
    beta = rng.standard_normal(4)
    z, att, br = orc.z_step(X, y, beta, 11, 4, chain=2)
    for i in range(50):
        eta = orc.row_dot(X, i, beta)
        zi, ai, bi = orc.tn_draw(eta, y[i], 11, i, 4, chain=2)
        assert zi == z[i] and ai == att[i] and bi == br[i]


def cheng_acceptance(a):
    lam = math.sqrt(2 * a - 1)
    return math.exp(special.gammaln(a) + math.log(lam) + a - math.log(4) - a * math.log(a))


@pytest.mark.parametrize("a", [1.5, 5.5, 50.5, 500.5])
def test_cheng_gamma(orc, a):
    n = 30_000
    g = np.empty(n)
    att = np.empty(n, np.int64)
    for k in range(n):
        g[k], att[k] = orc.gamma_cheng(a, 77, k + 1)
    assert abs(g.mean() - a) < 5 * math.sqrt(a / n)
    assert abs(g.var() / a - 1.0) < 6 * math.sqrt(2.0 / n) * math.sqrt(1 + 3 / a)
    assert stats.kstest(g, stats.gamma(a).cdf).pvalue > 1e-4
    acc = cheng_acceptance(a)
    first = np.mean(att == 0)
    assert abs(first - acc) < 5 * math.sqrt(acc * (1 - acc) / n)


def test_cheng_acceptance_matches_paper():
    """Section 5: about 0.88 per proposal; 32 proposals fail together ~3.4e-30."""
    for p in (100, 1000):
        acc = cheng_acceptance((p + 1) / 2)
        assert abs(acc - GOLD["cheng_per_proposal_acceptance"]["value"]) < 0.01
    fail = (1 - GOLD["cheng_per_proposal_acceptance"]["value"]) ** GOLD["cheng_block_threads"]["value"]
    assert abs(fail / GOLD["cheng_block_failure"]["value"] - 1) < 0.02


def test_exponential_draws(orc):
    p = 40_000
    rate_nu = 2.5
    # beta = 0 makes the lambda^-2 rate equal nu^-1
    lam, clamps = orc.lambda_step(np.zeros(p), np.full(p, rate_nu), 3.0, 5, 9)
    assert clamps == 0
    assert stats.kstest(lam, stats.expon(scale=1 / rate_nu).cdf).pvalue > 1e-4
    # rate nu^-1 + tau^-2 beta^2 / 2
    beta = np.full(p, 2.0)
    lam2, _ = orc.lambda_step(beta, np.full(p, 0.5), 0.25, 5, 10)
    assert stats.kstest(lam2, stats.expon(scale=1 / (0.5 + 0.25 * 4 / 2)).cdf).pvalue > 1e-4
    nu = orc.nu_step(np.full(p, 3.0), 5, 11)
    assert stats.kstest(nu, stats.expon(scale=1 / 4.0).cdf).pvalue > 1e-4
    xs = np.array([orc.xi_step(1.5, 5, k) for k in range(1, 20_001)])
    assert stats.kstest(xs, stats.expon(scale=1 / 2.5).cdf).pvalue > 1e-4


def test_lambda_rate_clamp(orc):
    lam, clamps = orc.lambda_step(np.zeros(3), np.zeros(3), 1.0, 1, 1)
    assert clamps == 3
    assert np.all(lam > 0)


def test_tau_step_is_gamma_over_rate(orc):
    """tau^-2 = G/rate with G ~ Gamma((p+1)/2, 1), rate = xi^-1 + sum lam^-2 beta^2 / 2."""
    p = 9
    lam = np.linspace(0.5, 2.0, p)
    beta = np.linspace(-1, 1, p)
    xi = 0.7
    rate = xi + 0.5 * np.sum(lam * beta**2)
    draws = np.array([orc.tau_step(lam, beta, xi, 3, k)[0] for k in range(1, 20_001)])
    assert stats.kstest(draws, stats.gamma((p + 1) / 2, scale=1 / rate).cdf).pvalue > 1e-4
