"""Pins of the oracle's target U(h), its gradient, H and the dH sum.

U is checked against the model's own generative densities (scipy.stats
normal log-densities of eqs. (1)-(3) with a stationary h_1), the gradient
against central finite differences of U, dH against a 40-digit mpmath
evaluation of H(h',p') - H(h,p), and the compensated sum against exact
rational arithmetic.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest
from scipy import stats

import oracle
import synth

TH = synth.THETA_STAR


def _data(T, seed=1):
    y, lr, h = synth.simulate_rsv(T, TH, seed)
    return y * y, lr, h


def model_logpdf(h, y2, r, th, terms=3):
    """log p(h, data | theta) straight from eqs. (1)-(3) + stationary h_1."""
    phi, mu, xi, se, su = (th[k] for k in ("phi", "mu", "xi", "sig2_eta", "sig2_u"))
    lp = stats.norm.logpdf(h[0], mu, np.sqrt(se / (1 - phi * phi)))
    lp += stats.norm.logpdf(h[1:], mu + phi * (h[:-1] - mu), np.sqrt(se)).sum()
    if terms & 1:
        lp += stats.norm.logpdf(np.sqrt(y2), 0.0, np.exp(0.5 * h)).sum()
    if terms & 2:
        lp += stats.norm.logpdf(r, xi + h, np.sqrt(su)).sum()
    return lp


@pytest.mark.parametrize("terms", [1, 2, 3])
def test_energy_is_negative_log_model_density(terms):
    y2, r, h_true = _data(300)
    rng = np.random.default_rng(3)
    ths = [TH, dict(phi=-0.4, mu=0.7, xi=-1.1, sig2_eta=0.3, sig2_u=0.02)]
    for th in ths:
        hs = [h_true, h_true + 0.3 * rng.standard_normal(300), r - th["xi"]]
        u = [oracle.energy(h, y2, r, th, terms) for h in hs]
        lp = [model_logpdf(h, y2, r, th, terms) for h in hs]
        for i in range(1, len(hs)):
            # U is -log density up to a constant that does not depend on h
            assert (u[i] - u[0]) == pytest.approx(-(lp[i] - lp[0]), rel=1e-10, abs=1e-9)


@pytest.mark.parametrize("terms", [1, 2, 3])
@pytest.mark.parametrize("T", [1, 2, 3, 64])
def test_gradient_matches_central_differences(terms, T):
    y2, r, h_true = _data(max(T, 3), seed=4)
    y2, r, h = y2[:T], r[:T], h_true[:T] + 0.1
    g = oracle.grad(h, y2, r, TH, terms)
    for t in range(T):
        eps = 1e-5 * max(1.0, abs(h[t]))
        hp, hm = h.copy(), h.copy()
        hp[t] += eps
        hm[t] -= eps
        fd = (oracle.energy(hp, y2, r, TH, terms) - oracle.energy(hm, y2, r, TH, terms)) / (2 * eps)
        assert abs(fd - g[t]) <= 1e-7 * max(1.0, abs(g[t])), (t, fd, g[t])


def test_gradient_long_series_spot_check():
    y2, r, h = _data(1000, seed=1)
    g = oracle.grad(h, y2, r, TH)
    for t in [0, 1, 2, 499, 997, 998, 999]:
        eps = 1e-5 * max(1.0, abs(h[t]))
        hp, hm = h.copy(), h.copy()
        hp[t] += eps
        hm[t] -= eps
        fd = (oracle.energy(hp, y2, r, TH) - oracle.energy(hm, y2, r, TH)) / (2 * eps)
        assert abs(fd - g[t]) <= 1e-7 * max(1.0, abs(g[t]))


def test_hamiltonian_kinetic_term_with_mass():
    y2, r, h = _data(50)
    rng = np.random.default_rng(0)
    p = rng.standard_normal(50)
    lm = 0.5 * rng.standard_normal(50)
    H1 = oracle.hamiltonian(h, p, y2, r, TH, log_m=lm)
    H0 = oracle.hamiltonian(h, np.zeros(50), y2, r, TH, log_m=lm)
    assert H1 - H0 == pytest.approx(np.sum(p * p / (2 * np.exp(lm))), rel=1e-12)


def _H_mp(h, p, y2, r, th, log_m=None):
    """H in 40-digit arithmetic from the model's normal densities (constants
    dropped: each density contributes its squared-residual term; eq. (1)
    also contributes its log-variance h_t/2)."""
    mpmath.mp.dps = 40
    f = mpmath.mpf
    phi, mu, xi, se, su = (f(th[k]) for k in ("phi", "mu", "xi", "sig2_eta", "sig2_u"))
    H = f(0)
    T = len(h)
    hs = [f(x) for x in h]
    for t in range(T):
        m = f(1) if log_m is None else mpmath.exp(f(log_m[t]))
        H += f(p[t]) ** 2 / (2 * m)
        H += hs[t] / 2 + f(y2[t]) * mpmath.exp(-hs[t]) / 2
        H += (f(r[t]) - xi - hs[t]) ** 2 / (2 * su)
    H += (1 - phi * phi) * (hs[0] - mu) ** 2 / (2 * se)
    for t in range(T - 1):
        H += ((hs[t + 1] - mu) - phi * (hs[t] - mu)) ** 2 / (2 * se)
    return H


@pytest.mark.parametrize("with_mass", [False, True])
def test_delta_h_matches_high_precision_difference(with_mass):
    T = 200
    y2, r, h0 = _data(T, seed=6)
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(T)
    lm = 0.3 * rng.standard_normal(T) if with_mass else None
    h1, p1 = oracle.leapfrog(h0, p0, y2, r, TH, k=20, dtau=0.05, log_m=lm)
    dH = oracle.delta_h(h0, p0, h1, p1, y2, r, TH, log_m=lm)
    ref = _H_mp(h1, p1, y2, r, TH, lm) - _H_mp(h0, p0, y2, r, TH, lm)
    assert abs(dH - float(ref)) <= 1e-12, (dH, float(ref))


def _exact_sum(x):
    return float(sum((Fraction(v) for v in x), Fraction(0)))


@pytest.mark.parametrize("seq", [
    [1.0, 1e100, 1.0, -1e100],
    [1e16, 1.0, -1e16, 3.0],
    [0.1] * 10 + [-1.0],
])
def test_neumaier_exact_on_classic_cases(seq):
    assert oracle.neumaier_sum(seq) == _exact_sum(seq)


def test_neumaier_within_bound_on_random_cancellation():
    rng = np.random.default_rng(2)
    eps = np.finfo(float).eps
    for _ in range(50):
        n = 2000
        x = rng.standard_normal(n) * 10.0 ** rng.integers(-8, 9, size=n)
        x = np.concatenate([x, -x[: n // 2] * (1 + 1e-12)])
        rng.shuffle(x)
        s = oracle.neumaier_sum(x)
        ex = _exact_sum(x)
        assert abs(s - ex) <= 2 * eps * abs(ex) + 4 * x.size * eps * eps * np.abs(x).sum()
