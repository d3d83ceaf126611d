"""Pins of the oracle's theta update (sufficient statistics + Gibbs/MH).

The paper states no priors and no theta sampler; the oracle's derivation
(closed-form Gaussian / inverse-Gamma conditionals from shifted sufficient
statistics, and an independence Metropolis step for phi) is checked here
against brute force: each conditional is re-derived numerically by 1-D
quadrature of prior x the model's own densities (scipy.stats, eqs. (1)-(3)
with a stationary h_1), evaluated on the raw h and data, and the oracle's
draws are tested by the probability integral transform (KS to U(0,1)).
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from tests._stats import bracket, grid_cdf

T = 50
TH = dict(synth.THETA_STAR)
PRIOR = dict(oracle.DEFAULT_PRIOR)
N_DRAWS = 1500


@pytest.fixture(scope="module")
def data():
    y, r, h = synth.simulate_rsv(T, TH, 21)
    return y * y, r, h


def log_h_given(h, mu, phi, s_eta):
    """log p(h | mu, phi, s_eta) for arrays of one varying parameter."""
    mu, phi, s_eta = np.broadcast_arrays(np.asarray(mu, float), np.asarray(phi, float),
                                         np.asarray(s_eta, float))
    out = stats.norm.logpdf(h[0], mu, np.sqrt(s_eta / (1 - phi ** 2)))
    hm = h[None, :] - mu.reshape(-1, 1)
    innov = hm[:, 1:] - phi.reshape(-1, 1) * hm[:, :-1]
    out = out.reshape(-1) + stats.norm.logpdf(innov, 0.0, np.sqrt(s_eta).reshape(-1, 1)).sum(1)
    return out


def log_r_given(h, r, xi, s_u):
    xi, s_u = np.broadcast_arrays(np.asarray(xi, float), np.asarray(s_u, float))
    res = r[None, :] - h[None, :] - xi.reshape(-1, 1)
    return stats.norm.logpdf(res, 0.0, np.sqrt(s_u).reshape(-1, 1)).sum(1)


def pit(draw, logpdf_vec, center, scale, positive=False):
    lo, hi = bracket(logpdf_vec, center, scale, positive=positive)
    xs, cdf = grid_cdf(logpdf_vec, lo, hi)
    return float(np.interp(draw, xs, cdf))


def run_updates(h, r, th_in, prior=PRIOR, n=N_DRAWS):
    st = oracle.suffstats(h, r, th_in["mu"], th_in["xi"])
    outs = []
    for i in range(n):
        th, flags = oracle.theta_update(T, st, th_in, seed=9, sweep=i, chain=3, prior=prior)
        assert not (flags & 2)
        outs.append(th)
    return outs


def test_suffstats_shift_invariance(data):
    """The statistics at two different shifts describe the same h: the
    implied raw sums must agree."""
    y2, r, h = data
    a = oracle.suffstats(h, r, 0.0, 0.0)
    c_mu, c_xi = -0.37, 0.21
    b = oracle.suffstats(h, r, c_mu, c_xi)
    assert b[0] == pytest.approx(a[0] - T * c_mu, rel=1e-13)
    assert b[1] == pytest.approx(a[1] - 2 * c_mu * a[0] + T * c_mu ** 2, rel=1e-13)
    assert b[3] == pytest.approx(a[3] - T * c_xi, rel=1e-13)
    assert b[5] == pytest.approx(h[0] - c_mu) and b[6] == pytest.approx(h[-1] - c_mu)


def test_mu_conditional(data):
    y2, r, h = data
    outs = run_updates(h, r, TH)
    lp = lambda m: (stats.norm.logpdf(m, PRIOR["mu_mean"], np.sqrt(PRIOR["mu_var"]))
                    + log_h_given(h, m, TH["phi"], TH["sig2_eta"]))
    lo, hi = bracket(lp, h.mean(), 0.5)
    xs, cdf = grid_cdf(lp, lo, hi)
    u = np.interp([o["mu"] for o in outs], xs, cdf)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_sig2_eta_conditional_given_new_mu_phi(data):
    y2, r, h = data
    outs = run_updates(h, r, TH, n=600)
    ig = stats.invgamma(PRIOR["eta_shape"], scale=PRIOR["eta_scale"])
    u = []
    for o in outs:
        lp = lambda s: ig.logpdf(s) + log_h_given(h, o["mu"], o["phi"], s)
        u.append(pit(o["sig2_eta"], lp, TH["sig2_eta"], 0.02, positive=True))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_xi_conditional(data):
    y2, r, h = data
    outs = run_updates(h, r, TH)
    lp = lambda x: (stats.norm.logpdf(x, PRIOR["xi_mean"], np.sqrt(PRIOR["xi_var"]))
                    + log_r_given(h, r, x, TH["sig2_u"]))
    lo, hi = bracket(lp, TH["xi"], 0.1)
    xs, cdf = grid_cdf(lp, lo, hi)
    u = np.interp([o["xi"] for o in outs], xs, cdf)
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_sig2_u_conditional_given_new_xi(data):
    y2, r, h = data
    outs = run_updates(h, r, TH, n=600)
    ig = stats.invgamma(PRIOR["u_shape"], scale=PRIOR["u_scale"])
    u = []
    for o in outs:
        lp = lambda s: ig.logpdf(s) + log_r_given(h, r, o["xi"], s)
        u.append(pit(o["sig2_u"], lp, TH["sig2_u"], 0.03, positive=True))
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_phi_metropolis_leaves_conditional_invariant(data):
    """Start phi from its exact conditional (inverse CDF on a grid) with mu
    pinned by a point-mass prior; one independence-MH step must return a
    draw from the same conditional."""
    y2, r, h = data
    lp = lambda p: log_h_given(h, TH["mu"], p, TH["sig2_eta"])
    xs, cdf = grid_cdf(lp, -1 + 1e-9, 1 - 1e-9, n=20001)
    rng = np.random.default_rng(4)
    pinned = dict(PRIOR, mu_mean=TH["mu"], mu_var=1e-16)
    n = 3000
    phi_in = np.interp(rng.uniform(size=n), cdf, xs)
    out, n_acc = [], 0
    for i in range(n):
        th_in = dict(TH, phi=float(phi_in[i]))
        st = oracle.suffstats(h, r, th_in["mu"], th_in["xi"])
        th, flags = oracle.theta_update(T, st, th_in, seed=13, sweep=i, chain=0, prior=pinned)
        assert abs(th["mu"] - TH["mu"]) < 1e-6
        out.append(th["phi"])
        n_acc += flags & 1
    u = np.interp(out, xs, cdf)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert n_acc > 0.3 * n


def test_rv_term_off_keeps_xi_and_sig2_u(data):
    y2, r, h = data
    st = oracle.suffstats(h, r, TH["mu"], TH["xi"])
    th, _ = oracle.theta_update(T, st, TH, seed=1, sweep=0, chain=0, terms=oracle.TERM_RETURN)
    assert th["xi"] == TH["xi"] and th["sig2_u"] == TH["sig2_u"]
    assert th["mu"] != TH["mu"]
