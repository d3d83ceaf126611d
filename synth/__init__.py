"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module simulates the RSV model forward to make data; it holds none of
the sampler's arithmetic (no target, force, integrator or update).  Every
draw comes from numpy's PCG64 seeded by the caller.

Model (Takaishi, arXiv:1603.08114, Sec. 2, eqs. (1)-(3)):
    y_t       = exp(h_t/2) eps_t,            eps_t ~ N(0,1)
    ln RV_t   = xi + h_t + u_t,              u_t   ~ N(0, sigma_u^2)
    h_{t+1}   = mu + phi (h_t - mu) + eta_t, eta_t ~ N(0, sigma_eta^2)
with h_1 drawn from the stationary law N(mu, sigma_eta^2 / (1 - phi^2)).
"""
from __future__ import annotations

import numpy as np

THETA_KEYS = ("phi", "mu", "xi", "sig2_eta", "sig2_u")

# Parameter set of the single-series workloads (phi, mu, xi, s_eta, s_u).
THETA_STAR = dict(phi=0.97, mu=-0.3, xi=-0.2, sig2_eta=0.04, sig2_u=0.09)

# Ranges of the per-series parameters of the batched workloads.
BATCH_THETA_RANGES = dict(phi=(0.90, 0.99), mu=(-1.0, 0.5), xi=(-0.4, 0.0),
                          sig2_eta=(0.01, 0.1), sig2_u=(0.03, 0.2))


def simulate_rsv(T: int, theta: dict, seed: int):
    """One series of length T.  Returns (y, log_rv, h_true), float64."""
    rng = np.random.default_rng(seed)
    phi, mu, xi = theta["phi"], theta["mu"], theta["xi"]
    s_eta, s_u = np.sqrt(theta["sig2_eta"]), np.sqrt(theta["sig2_u"])
    eta = rng.standard_normal(T)
    h = np.empty(T)
    h[0] = mu + eta[0] * s_eta / np.sqrt(1.0 - phi * phi)
    for t in range(1, T):
        h[t] = mu + phi * (h[t - 1] - mu) + s_eta * eta[t]
    eps = rng.standard_normal(T)
    u = rng.standard_normal(T)
    y = np.exp(0.5 * h) * eps
    log_rv = xi + h + s_u * u
    return y, log_rv, h


def simulate_rsv_long(T: int, theta: dict, seed: int):
    """Same law as simulate_rsv for long T, with the AR(1) recursion run by
    scipy's linear filter.  Returns (y, log_rv, h_true)."""
    from scipy.signal import lfilter
    rng = np.random.default_rng(seed)
    phi, mu, xi = theta["phi"], theta["mu"], theta["xi"]
    s_eta, s_u = np.sqrt(theta["sig2_eta"]), np.sqrt(theta["sig2_u"])
    eta = rng.standard_normal(T)
    drive = s_eta * eta
    drive[0] = eta[0] * s_eta / np.sqrt(1.0 - phi * phi)
    h = lfilter([1.0], [1.0, -phi], drive) + mu
    eps = rng.standard_normal(T)
    u = rng.standard_normal(T)
    y = np.exp(0.5 * h) * eps
    log_rv = xi + h + s_u * u
    return y, log_rv, h


def draw_batch_thetas(n_series: int, seed: int):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_series):
        out.append({k: float(rng.uniform(*BATCH_THETA_RANGES[k])) for k in THETA_KEYS})
    return out


def make_batch(n_series: int, T_lo: int, T_hi: int, seed: int):
    """Batched workload: T_s ~ U{T_lo..T_hi}, per-series theta from the ranges.

    Returns dict(offsets int64[S+1], y, log_rv (concatenated), h_true, thetas).
    """
    rng = np.random.default_rng(seed)
    Ts = rng.integers(T_lo, T_hi + 1, size=n_series)
    thetas = draw_batch_thetas(n_series, seed + 1_000_003)
    ys, rvs, hs = [], [], []
    for s in range(n_series):
        y, lr, h = simulate_rsv_long(int(Ts[s]), thetas[s], seed * 7919 + s)
        ys.append(y); rvs.append(lr); hs.append(h)
    offsets = np.zeros(n_series + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(Ts)
    return dict(offsets=offsets, y=np.concatenate(ys), log_rv=np.concatenate(rvs),
                h_true=np.concatenate(hs), thetas=thetas)


def theta_array(thetas):
    """List of theta dicts -> float64 array [n, 5] in (phi, mu, xi, s_eta, s_u) order."""
    if isinstance(thetas, dict):
        thetas = [thetas]
    return np.array([[t[k] for k in THETA_KEYS] for t in thetas], dtype=np.float64)
