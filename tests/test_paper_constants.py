"""Pins from numbers the paper prints (tests/golden/paper_constants.json).

* The cold start of Section 6.1, as the oracle's orc_cold_start sets it.
* The synthetic design of Eq. (13): its leading coefficients, and that the
  oracle's posterior on such data recovers them (Section 6.1 reports the
  truth is recovered).
* The memory figure of Section 6.1: a float32 design with N = 1,000,000 and
  p = 10,000 takes over 40 GB.
"""
import json
import os

import numpy as np

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_cold_start_is_the_papers(orc):
    g = GOLD["cold_start"]
    c = orc.Chain(7)
    assert np.all(c.beta == g["beta"])
    assert np.all(c.lam_m2 == g["lambda"] ** -2) and np.all(c.nu_m1 == g["nu"] ** -1)
    assert c.tau_m2 == g["tau"] ** -2 and c.xi_m1 == g["xi"] ** -1 and c.sweep == 0


def test_eq13_design_and_recovery(orc):
    lead = np.array(GOLD["eq13_beta"]["value"])
    d = synth.eq13(3000, 12, seed=21)
    assert np.array_equal(d.beta_true[:6], lead) and np.all(d.beta_true[6:] == 0.0)
    assert not d.intercept and np.all(d.X[:, 0] != 1.0)
    G = orc.gram(d.X)
    c = orc.Chain(d.p)
    beta, _ = c.run(d.X, d.y, G, seed=3, n=1500)
    post = beta[300:]
    mean, sd = post.mean(0), post.std(0)
    # every nonzero coefficient lies within 4 posterior standard deviations of
    # the posterior mean, which is itself clearly away from 0
    assert np.all(np.abs(mean[:6] - lead) <= 4 * sd[:6])
    assert np.all(np.sign(mean[:6]) == np.sign(lead)) and np.all(np.abs(mean[:6]) > 4 * sd[:6])
    # the zero coefficients are shrunk towards 0
    assert np.all(np.abs(mean[6:]) < 0.25)


def test_memory_of_the_design_the_paper_could_not_run():
    g = GOLD["x_bytes_1e6_by_1e4"]
    N, p = g["N"], g["p"]
    assert N * p * 4 + N >= g["value_gb_lower_bound"] * 1e9


def test_rare_event_stand_in_has_the_papers_shape():
    """The synthetic stand-in for the Section 6.2 data has its shape and its
    outcome rate (the data themselves are not available)."""
    g = GOLD["real_data_shape"]
    assert (synth.RARE_N, synth.RARE_P, synth.RARE_YBAR) == (g["N"], g["p"], g["ybar"])
    d = synth.rare_event(N=200_000)
    assert d.p == g["p"] and np.all(d.X[:, 0] == 1.0)
    assert abs(d.y.mean() / g["ybar"] - 1.0) < 0.1
