"""Small statistics helpers for the statistical pins (test-only)."""
import numpy as np


def batch_means_mcse(x, n_batches=None):
    """Monte Carlo standard error of the mean of each column of x (n, ...)
    by non-overlapping batch means with floor(sqrt(n)) batches."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    b = n_batches or int(np.floor(np.sqrt(n)))
    m = n // b
    xb = x[: b * m].reshape((b, m) + x.shape[1:]).mean(axis=1)
    return xb.std(axis=0, ddof=1) / np.sqrt(b)


def z_scores_mean_var(draws, ref_mean, ref_var):
    """z of posterior mean and variance of each column against exact values."""
    draws = np.asarray(draws)
    m = draws.mean(axis=0)
    se_m = batch_means_mcse(draws)
    dev2 = (draws - m) ** 2
    v = dev2.mean(axis=0)
    se_v = batch_means_mcse(dev2)
    return (m - ref_mean) / se_m, (v - ref_var) / se_v


def z_rule_ok(z):
    """Multiple-comparison rule over N quantities: the share with |z| > 3 is
    at most 0.27% + 3 sd of that share, and max |z| <= sqrt(2 ln N) + 1."""
    z = np.abs(np.ravel(z))
    N = z.size
    frac_limit = 0.0027 + 3.0 * np.sqrt(0.0027 * 0.9973 / N)
    max_limit = np.sqrt(2.0 * np.log(max(N, 2))) + 1.0
    return (np.mean(z > 3.0) <= frac_limit) and (z.max() <= max(max_limit, 3.0))


def grid_cdf(logpdf_vec, lo, hi, n=8001):
    """CDF of an unnormalised 1-D log density (vectorised) on [lo, hi]."""
    xs = np.linspace(lo, hi, n)
    lp = logpdf_vec(xs)
    w = np.exp(lp - np.nanmax(lp))
    w = np.where(np.isfinite(w), w, 0.0)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (w[1:] + w[:-1]) * np.diff(xs))])
    return xs, cdf / cdf[-1]


def bracket(logpdf_vec, center, scale, drop=40.0, positive=False):
    """Interval around `center` outside which the log density is `drop`
    below its maximum (grows the interval until it is)."""
    lo, hi = center - 10 * scale, center + 10 * scale
    if positive:
        lo = max(lo, 1e-12)
    for _ in range(60):
        xs = np.linspace(lo, hi, 2001)
        lp = logpdf_vec(xs)
        mx = np.nanmax(lp)
        ok_lo = lp[0] < mx - drop or (positive and lo <= 1e-12)
        ok_hi = lp[-1] < mx - drop
        if ok_lo and ok_hi:
            return lo, hi
        w = hi - lo
        if not ok_lo:
            lo = lo - w if not positive else max(lo - w, 1e-12)
        if not ok_hi:
            hi = hi + w
    return lo, hi
