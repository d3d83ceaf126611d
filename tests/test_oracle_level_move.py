"""Pins of the oracle's level move (h -> h + c, mu -> mu + c, xi -> xi - c).

Along that orbit the joint posterior of (h, theta) reduces to the return
likelihood prod_t N(y_t; 0, e^{h_t + c}) times the priors of mu + c and
xi - c (the AR(1) part depends on h - mu and the RV residuals on
r - xi - h, both unchanged).  Repeated moves from one state therefore walk
the orbit with that density as their stationary law.  The tests build the
density here from scipy's normal log densities on a grid, independently of
the oracle, and compare the walk's positions with it:
* vague priors: the move is an exact draw (acceptance ~1), positions are
  independent -> Kolmogorov-Smirnov against the grid CDF;
* tight priors: the Metropolis correction matters -> mean and variance of
  the positions within 4 batch-means standard errors of the grid moments;
* RV term only: c is Gaussian from the two prior factors.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from tests._stats import batch_means_mcse

TH = dict(synth.THETA_STAR)


def orbit_density(y, h, th, prior, terms, grid):
    lp = np.zeros_like(grid)
    if terms & oracle.TERM_RETURN:
        for t in range(h.size):
            lp += stats.norm.logpdf(y[t], 0.0, np.exp(0.5 * (h[t] + grid)))
    lp += stats.norm.logpdf(th["mu"] + grid, prior["mu_mean"], np.sqrt(prior["mu_var"]))
    if terms & oracle.TERM_RV:
        lp += stats.norm.logpdf(th["xi"] - grid, prior["xi_mean"], np.sqrt(prior["xi_var"]))
    w = np.exp(lp - lp.max())
    return w / np.trapezoid(w, grid)


def walk(h, th, y2, prior, terms, n, seed=3):
    pos = np.empty(n)
    total = 0.0
    acc = 0
    for i in range(n):
        out = oracle.level_move(h, th, y2, seed, i, 0, prior=prior, terms=terms)
        h, th = out["h"], out["theta"]
        total += out["c"]
        acc += bool(out["flags"] & 2)
        pos[i] = total
    return pos, acc / n, h, th


def _state(T, seed):
    y, r, h = synth.simulate_rsv(T, TH, seed)
    return y, r, h


def test_vague_prior_walk_matches_orbit_density_ks():
    y, r, h = _state(40, 11)
    prior = dict(oracle.DEFAULT_PRIOR)
    pos, acc, h_end, th_end = walk(h, dict(TH), y * y, prior, oracle.TERMS_RSV, 6000)
    assert acc > 0.99
    # every move is one translation of h, mu and xi by the same c
    np.testing.assert_allclose(h_end - h, pos[-1], atol=1e-9)
    assert th_end["mu"] - TH["mu"] == pytest.approx(pos[-1], abs=1e-9)
    assert th_end["xi"] - TH["xi"] == pytest.approx(-pos[-1], abs=1e-9)
    for k in ("phi", "sig2_eta", "sig2_u"):
        assert th_end[k] == TH[k]
    grid = np.linspace(-3.0, 3.0, 24001)
    dens = orbit_density(y, h, TH, prior, oracle.TERMS_RSV, grid)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (dens[1:] + dens[:-1]) * np.diff(grid))])
    assert cdf[-1] == pytest.approx(1.0, abs=1e-6) and dens[0] < 1e-12 and dens[-1] < 1e-12
    ks = stats.kstest(pos, lambda x: np.interp(x, grid, cdf))
    assert ks.pvalue > 1e-3, ks


@pytest.mark.parametrize("terms", [oracle.TERMS_RSV, oracle.TERM_RETURN])
def test_tight_prior_walk_matches_orbit_moments(terms):
    y, r, h = _state(40, 12)
    prior = dict(oracle.DEFAULT_PRIOR, mu_mean=-0.1, mu_var=0.02, xi_mean=-0.5, xi_var=0.03)
    pos, acc, _, _ = walk(h, dict(TH), y * y, prior, terms, 40000, seed=5)
    assert 0.05 < acc < 0.95  # the prior test is doing work
    grid = np.linspace(-3.0, 3.0, 24001)
    dens = orbit_density(y, h, TH, prior, terms, grid)
    m = np.trapezoid(grid * dens, grid)
    v = np.trapezoid((grid - m) ** 2 * dens, grid)
    draws = pos[500:]
    assert abs(draws.mean() - m) <= 4 * batch_means_mcse(draws), (draws.mean(), m)
    dev2 = (draws - draws.mean()) ** 2
    assert abs(dev2.mean() - v) <= 4 * batch_means_mcse(dev2), (dev2.mean(), v)


def test_rv_only_level_is_gaussian_prior_part():
    y, r, h = _state(30, 13)
    prior = dict(oracle.DEFAULT_PRIOR, mu_mean=0.3, mu_var=0.5, xi_mean=-0.2, xi_var=0.25)
    pos, acc, _, _ = walk(h, dict(TH), y * y, prior, oracle.TERM_RV, 8000, seed=6)
    assert acc == 1.0
    # N(mu + c; m_mu, v_mu) N(xi - c; m_xi, v_xi) in c: precision 1/v_mu + 1/v_xi
    prec = 1 / 0.5 + 1 / 0.25
    mean = ((0.3 - TH["mu"]) / 0.5 + (TH["xi"] + 0.2) / 0.25) / prec
    ks = stats.kstest(pos, stats.norm(mean, 1 / np.sqrt(prec)).cdf)
    assert ks.pvalue > 1e-3, ks
