"""Statistical pins of the oracle's whole h-sampler (theta held fixed).

The trajectories here are kept short (k dtau = 0.25, below half a period of
the stiffest Gaussian mode) so that the fixed-length sampler is ergodic in
every mode and batch-means standard errors are valid; at k dtau near a
multiple of pi/omega a Gaussian mode of frequency omega barely moves.

* Linear-Gaussian case (eq. (1) dropped): the exact posterior of h is
  Gaussian; its means and variances come from a Kalman filter + RTS smoother
  and, independently, from the tridiagonal posterior precision.  HMC moments
  must agree within Monte Carlo error (z-rule over sites).
* Full RSV target at T = 2 and T = 3: E[h_t] and Var[h_t] by brute-force
  tensor-product quadrature of the model density.
* Creutz identity <exp(-dH)> = 1 at equilibrium.
"""
import numpy as np
import pytest
from scipy import stats

import oracle
import synth
from tests._stats import batch_means_mcse, z_rule_ok, z_scores_mean_var

TH = dict(synth.THETA_STAR)


def kalman_rts(z, phi, s_eta, s_u):
    """Posterior mean/var of a_t given z_t = a_t + u_t, a_1 stationary."""
    T = z.size
    mp = np.zeros(T); Pp = np.zeros(T); mf = np.zeros(T); Pf = np.zeros(T)
    mp[0], Pp[0] = 0.0, s_eta / (1 - phi * phi)
    for t in range(T):
        if t > 0:
            mp[t] = phi * mf[t - 1]
            Pp[t] = phi * phi * Pf[t - 1] + s_eta
        K = Pp[t] / (Pp[t] + s_u)
        mf[t] = mp[t] + K * (z[t] - mp[t])
        Pf[t] = (1 - K) * Pp[t]
    ms, Ps = mf.copy(), Pf.copy()
    for t in range(T - 2, -1, -1):
        G = Pf[t] * phi / Pp[t + 1]
        ms[t] = mf[t] + G * (ms[t + 1] - mp[t + 1])
        Ps[t] = Pf[t] + G * G * (Ps[t + 1] - Pp[t + 1])
    return ms, Ps


def tridiag_posterior(z, phi, s_eta, s_u):
    T = z.size
    Q = np.diag(np.full(T, 1 + phi * phi)) - phi * (np.eye(T, k=1) + np.eye(T, k=-1))
    Q[0, 0] = Q[-1, -1] = 1.0
    prec = Q / s_eta + np.eye(T) / s_u
    cov = np.linalg.inv(prec)
    return cov @ (z / s_u), np.diag(cov)


@pytest.mark.parametrize("with_mass", [False, True])
def test_linear_gaussian_matches_kalman_smoother(with_mass):
    T = 50
    y, r, h_true = synth.simulate_rsv(T, TH, 31)
    y2 = y * y
    z = r - TH["xi"] - TH["mu"]
    km, kv = kalman_rts(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    tm, tv = tridiag_posterior(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    np.testing.assert_allclose(km, tm, rtol=0, atol=1e-12)
    np.testing.assert_allclose(kv, tv, rtol=1e-12)
    lm, k, dtau = None, 5, 0.05
    if with_mass:
        lm, k, dtau = 0.3 * np.random.default_rng(2).standard_normal(T), 4, 0.04
    out = oracle.run(h_true, TH, y2, r, k=k, dtau=dtau, n_sweeps=100_000, seed=5,
                     update_theta=False, terms=oracle.TERM_RV, log_m=lm, keep_h=True)
    assert out["accepted"].mean() > 0.6
    draws = out["h_trace"][1000:]
    zm, zv = z_scores_mean_var(draws, km + TH["mu"], kv)
    assert z_rule_ok(zm), zm
    assert z_rule_ok(zv), zv


def _quadrature_moments(T, y2, r, th, n):
    # grid centred on the linear-Gaussian posterior, +-9 of its sd
    z = r - th["xi"] - th["mu"]
    m0, v0 = tridiag_posterior(z, th["phi"], th["sig2_eta"], th["sig2_u"])
    axes = [np.linspace(m0[t] + th["mu"] - 9 * np.sqrt(v0[t]),
                        m0[t] + th["mu"] + 9 * np.sqrt(v0[t]), n) for t in range(T)]
    grids = np.meshgrid(*axes, indexing="ij")
    H = [g.ravel() for g in grids]
    phi, mu, xi = th["phi"], th["mu"], th["xi"]
    lp = stats.norm.logpdf(H[0], mu, np.sqrt(th["sig2_eta"] / (1 - phi * phi)))
    for t in range(T):
        lp += stats.norm.logpdf(np.sqrt(y2[t]), 0.0, np.exp(0.5 * H[t]))
        lp += stats.norm.logpdf(r[t], xi + H[t], np.sqrt(th["sig2_u"]))
        if t + 1 < T:
            lp += stats.norm.logpdf(H[t + 1], mu + phi * (H[t] - mu), np.sqrt(th["sig2_eta"]))
    w = np.exp(lp - lp.max())
    w /= w.sum()
    mean = np.array([np.sum(w * H[t]) for t in range(T)])
    var = np.array([np.sum(w * (H[t] - mean[t]) ** 2) for t in range(T)])
    # the grid must hold essentially all the mass
    edge = np.zeros(grids[0].shape, bool)
    for ax in range(T):
        sl = [slice(None)] * T
        sl[ax] = 0
        edge[tuple(sl)] = True
        sl[ax] = -1
        edge[tuple(sl)] = True
    assert w.reshape(grids[0].shape)[edge].sum() < 1e-10
    return mean, var


@pytest.mark.parametrize("T,n_grid", [(2, 401), (3, 161)])
def test_small_T_full_target_matches_quadrature(T, n_grid):
    y, r, _ = synth.simulate_rsv(T, TH, 40 + T)
    y2 = y * y
    y2[0] *= 6.0  # a large return so the exp(-h) term matters
    qm, qv = _quadrature_moments(T, y2, r, TH, n_grid)
    out = oracle.run(r - TH["xi"], TH, y2, r, k=5, dtau=0.05, n_sweeps=200_000, seed=7,
                     update_theta=False, keep_h=True)
    draws = out["h_trace"][2000:]
    zm, zv = z_scores_mean_var(draws, qm, qv)
    assert np.all(np.abs(zm) <= 3.5), (zm, draws.mean(0), qm)
    assert np.all(np.abs(zv) <= 3.5), (zv, draws.var(0), qv)


def test_creutz_identity():
    T = 1000
    y, r, h = synth.simulate_rsv(T, TH, 1)
    out = oracle.run(h, TH, y * y, r, k=20, dtau=0.05, n_sweeps=3000, seed=3,
                     update_theta=False)
    e = np.exp(-out["dH"][200:])
    mcse = batch_means_mcse(e)
    assert abs(e.mean() - 1.0) <= 3 * mcse, (e.mean(), mcse)


def test_step_size_jitter_is_uniform_and_independent():
    """dtau_i / dtau - 1 over sweeps is U(-j, j) (Kolmogorov-Smirnov), chains
    draw independent factors, and j = 0 returns dtau exactly."""
    j, dtau, n = 0.3, 0.05, 20000
    f = np.array([oracle.step_size(9, s, 0, dtau, j) for s in range(n)]) / dtau - 1.0
    assert np.all(np.abs(f) <= j)
    assert stats.kstest(f, stats.uniform(loc=-j, scale=2 * j).cdf).pvalue > 1e-3
    g = np.array([oracle.step_size(9, s, 1, dtau, j) for s in range(n)]) / dtau - 1.0
    assert abs(np.corrcoef(f, g)[0, 1]) < 4.0 / np.sqrt(n)
    assert all(oracle.step_size(9, s, 0, dtau, 0.0) == dtau for s in range(100))


def test_jittered_long_trajectories_match_kalman_smoother():
    """k dtau = 1 puts several Gaussian modes of the linear-Gaussian target
    near a multiple of their half period, where a fixed-length sampler barely
    moves them; with the step size jittered by +-50% every mode mixes and the
    moments match the exact smoother (stationarity of the jittered chain)."""
    T = 50
    y, r, h_true = synth.simulate_rsv(T, TH, 31)
    z = r - TH["xi"] - TH["mu"]
    km, kv = kalman_rts(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    out = oracle.run(h_true, TH, y * y, r, k=20, dtau=0.05, n_sweeps=60_000, seed=6,
                     update_theta=False, terms=oracle.TERM_RV, keep_h=True, jitter=0.5)
    assert out["accepted"].mean() > 0.6
    draws = out["h_trace"][1000:]
    zm, zv = z_scores_mean_var(draws, km + TH["mu"], kv)
    assert z_rule_ok(zm), zm
    assert z_rule_ok(zv), zv
