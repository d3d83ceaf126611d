"""Effective sample size and Monte Carlo standard errors of MCMC output.

Host-side analysis of chains produced by the sampler (numpy only):

* ``ess_geyer`` -- Geyer's initial monotone sequence estimator (Geyer 1992,
  "Practical Markov chain Monte Carlo", Statist. Sci. 7): autocovariances by
  FFT, sums of adjacent pairs Gamma_k = gamma_{2k} + gamma_{2k+1} truncated at
  the first non-positive pair and forced monotone; tau = -1 + 2 sum Gamma_k.
* ``ess_batch_means`` -- from the means of b non-overlapping batches (for
  runs too long to store, accumulated on the device).
"""
from __future__ import annotations

import numpy as np


def _autocov(x: np.ndarray) -> np.ndarray:
    """Autocovariances (biased, divided by n) of each column, lags 0..n-1."""
    n = x.shape[0]
    xc = x - x.mean(axis=0)
    m = 1 << int(np.ceil(np.log2(2 * n)))
    f = np.fft.rfft(xc, n=m, axis=0)
    ac = np.fft.irfft(f * np.conj(f), n=m, axis=0)[:n]
    return ac / n


def integrated_time(x) -> np.ndarray:
    """Integrated autocorrelation time of each column (initial monotone sequence)."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    n, d = x.shape
    g = _autocov(x)
    tau = np.empty(d)
    for j in range(d):
        g0 = g[0, j]
        if g0 <= 0:
            tau[j] = np.nan
            continue
        npair = (n - 1) // 2
        pairs = g[0:2 * npair:2, j] + g[1:2 * npair + 1:2, j]
        pos = np.nonzero(pairs <= 0)[0]
        m = pos[0] if pos.size else npair
        p = np.minimum.accumulate(pairs[:m]) if m > 0 else pairs[:0]
        tau[j] = (-g0 + 2.0 * p.sum()) / g0
        tau[j] = max(tau[j], 1.0 / n)
    return tau


def ess_geyer(x) -> np.ndarray:
    """ESS of each column of draws x (n, d) or (n,)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    return n / integrated_time(x)


def ess_batch_means(batch_means, variance, n_draws: int) -> np.ndarray:
    """ESS from b batch means (b, d) of equal-length batches, the variance of
    the draws (d,) and the number of draws: ESS = var / MCSE^2 with
    MCSE^2 = var(batch means) / b."""
    bm = np.asarray(batch_means, dtype=np.float64)
    b = bm.shape[0]
    s2 = bm.var(axis=0, ddof=1)
    mcse2 = s2 / b
    with np.errstate(divide="ignore", invalid="ignore"):
        ess = np.asarray(variance) / mcse2
    return np.minimum(ess, n_draws * 10.0)


def mcse_mean(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    return np.sqrt(x.var(axis=0) / ess_geyer(x))


# --- comparing two samplers' posterior moments -----------------------------------
# Each side runs k independent chains from the same start; the moments of a
# quantity are the grand mean of its per-chain means (or variances), with a
# standard error from the chain-to-chain spread.  That error needs no model
# of the autocorrelation, and the comparison holds before convergence too:
# two correct implementations of one Markov kernel (or two exact kernels at
# equilibrium) give the same distribution of the chain state after each
# sweep from the same start.

def spread_summary(per_chain) -> tuple:
    """Grand mean, its standard error and the number of chains, from per-chain
    values (k, d) of a statistic."""
    v = np.asarray(per_chain, dtype=np.float64)
    k = v.shape[0]
    return v.mean(axis=0), v.std(axis=0, ddof=1) / np.sqrt(k), k


def welch_p(per_chain_a, per_chain_b):
    """Two-sided Welch-t p-values (and z) for equal grand means of a statistic
    per quantity, from per-chain values (k_a, d) and (k_b, d).  A quantity
    that no chain of either side moves (a parameter held fixed) has no
    spread: equal values give z = 0, p = 1; different values z = +-inf,
    p = 0."""
    from scipy import stats
    ma, sa, ka = spread_summary(per_chain_a)
    mb, sb, kb = spread_summary(per_chain_b)
    va, vb = sa * sa, sb * sb
    se = np.sqrt(va + vb)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = (ma - mb) / se
        df = (va + vb) ** 2 / (va * va / (ka - 1) + vb * vb / (kb - 1))
    a = np.asarray(per_chain_a, dtype=np.float64)
    b = np.asarray(per_chain_b, dtype=np.float64)
    fixed = (np.ptp(a, axis=0) == 0.0) & (np.ptp(b, axis=0) == 0.0)
    z = np.where(fixed, np.where(a[0] == b[0], 0.0, np.sign(a[0] - b[0]) * np.inf), z)
    p = 2.0 * stats.t.sf(np.abs(z), np.where(np.isfinite(df), df, ka + kb - 2))
    return z, p


def moment_rule(p, alpha_family=0.01, tail=0.0027):
    """The multiple-comparison rule for N quantities compared at once: the
    fraction of p-values below `tail` (the two-sided 3-sigma level) may
    exceed `tail` by at most three binomial standard errors, and the smallest
    p-value must be at least alpha_family / N (Bonferroni).  Returns
    (passed, summary)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    p = p[np.isfinite(p)]
    n = p.size
    frac = float(np.mean(p < tail))
    limit = tail + 3.0 * np.sqrt(tail * (1.0 - tail) / n)
    p_min = float(p.min())
    ok = frac <= limit and p_min >= alpha_family / n
    return ok, {"n": int(n), "frac_p_below_0.0027": frac, "frac_limit": float(limit),
                "min_p": p_min, "min_p_limit": alpha_family / n}
