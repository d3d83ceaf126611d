"""ESS estimators against AR(1) series of known integrated autocorrelation
time tau = (1 + rho) / (1 - rho)."""
import numpy as np
import pytest
from scipy.signal import lfilter

from paper_1603_08114_amd import diagnostics as D


def ar1(n, rho, d, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal((n, d))
    x = lfilter([1.0], [1.0, -rho], e, axis=0)
    return x[1000:]


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9, 0.99])
def test_geyer_integrated_time_ar1(rho):
    tau_true = (1 + rho) / (1 - rho)
    x = ar1(400_000 + 1000, rho, 8, seed=int(rho * 100))
    tau = D.integrated_time(x)
    assert np.all(np.abs(tau / tau_true - 1) < 0.10), (tau, tau_true)


def test_geyer_negative_correlation():
    # rho < 0: tau < 1, ESS > n (antithetic draws), still estimated
    x = ar1(200_000 + 1000, -0.5, 4, seed=3)
    tau = D.integrated_time(x)
    assert np.all(np.abs(tau / (1 / 3) - 1) < 0.15), tau


@pytest.mark.parametrize("rho", [0.5, 0.9])
def test_batch_means_ess_ar1(rho):
    n = 400_000
    x = ar1(n + 1000, rho, 16, seed=11)
    b = int(np.sqrt(n))
    m = n // b
    bm = x[: b * m].reshape(b, m, -1).mean(axis=1)
    ess = D.ess_batch_means(bm, x.var(axis=0), n)
    ess_true = n * (1 - rho) / (1 + rho)
    # batch-means ESS has ~ sqrt(2/b) relative scatter per column
    assert abs(np.median(ess) / ess_true - 1) < 0.1


def test_moment_rule_holds_under_the_null_and_catches_a_shift():
    """Per-chain means of 16 + 16 independent chains of an AR(1) process for
    4000 quantities: under equal means the rule passes (at its stated 1%
    family level it rarely fails: checked over 20 repetitions), and a shift of
    5 standard errors in 1% of the quantities fails it."""
    rng = np.random.default_rng(7)
    fails = 0
    for rep in range(20):
        a = rng.standard_normal((16, 4000))
        b = rng.standard_normal((16, 4000)) * 1.3 + 0.0
        _, p = D.welch_p(a, b)
        ok, _ = D.moment_rule(p)
        fails += not ok
    assert fails <= 1
    a = rng.standard_normal((16, 4000))
    b = rng.standard_normal((16, 4000))
    b[:, :40] += 5.0 * np.sqrt(2.0 / 16)
    _, p = D.welch_p(a, b)
    ok, summary = D.moment_rule(p)
    assert not ok, summary


def test_welch_p_matches_scipy_ttest():
    from scipy import stats
    rng = np.random.default_rng(3)
    a = rng.standard_normal((16, 5)) + 0.2
    b = rng.standard_normal((12, 5)) * 2.0
    _, p = D.welch_p(a, b)
    ref = stats.ttest_ind(a, b, axis=0, equal_var=False).pvalue
    np.testing.assert_allclose(p, ref, rtol=1e-10)


def test_welch_p_fixed_quantity():
    """A quantity constant over every chain of both sides: equal -> p = 1,
    different -> p = 0; the other quantities are unaffected."""
    rng = np.random.default_rng(3)
    a = np.column_stack([rng.standard_normal(16), np.full(16, 0.2), np.full(16, 0.1)])
    b = np.column_stack([rng.standard_normal(16), np.full(16, 0.2), np.full(16, 0.3)])
    z, p = D.welch_p(a, b)
    assert np.isfinite(z[0]) and 0.0 < p[0] <= 1.0
    assert z[1] == 0.0 and p[1] == 1.0
    assert np.isinf(z[2]) and p[2] == 0.0
