"""Pins of the oracle's Omelyan integrator (second-order minimum-norm,
h-first form; Omelyan, Mryglod and Folk 2003).

Properties fixed by the mathematics, each broken by a plausible slip (a
wrong coefficient, a kick at the wrong h, an asymmetric split):
* on the linear-Gaussian target (eq. (1) dropped) the exact Hamiltonian flow
  is a matrix exponential of the posterior precision; the integrator
  converges to it with order 2 and, at equal step size, more closely than
  the leapfrog;
* time reversibility and symplecticity (J^T Omega J = Omega) on the full
  RSV target, with and without a diagonal mass;
* the whole sampler at fixed theta reproduces the Kalman-smoother posterior.
"""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth
from tests._stats import z_rule_ok, z_scores_mean_var
from tests.test_oracle_posterior import kalman_rts, tridiag_posterior

TH = dict(synth.THETA_STAR)


def _data(T, seed=1):
    y, lr, h = synth.simulate_rsv(T, TH, seed)
    return y * y, lr, h


@pytest.mark.parametrize("with_mass", [False, True])
def test_reversibility(with_mass):
    T = 1000
    y2, r, h0 = _data(T)
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(T)
    lm = 0.4 * rng.standard_normal(T) if with_mass else None
    h1, p1 = oracle.omelyan(h0, p0, y2, r, TH, 10, 0.1, log_m=lm)
    assert np.max(np.abs(h1 - h0)) > 1e-2  # it moved
    h2, p2 = oracle.omelyan(h1, -p1, y2, r, TH, 10, 0.1, log_m=lm)
    assert np.max(np.abs(h2 - h0)) <= 1e-12 * max(1.0, np.max(np.abs(h0)))
    assert np.max(np.abs(-p2 - p0)) <= 1e-12 * max(1.0, np.max(np.abs(p0)))


@pytest.mark.parametrize("with_mass", [False, True])
def test_symplectic_T3(with_mass):
    T = 3
    y2, r, h0 = _data(T, seed=2)
    p0 = np.array([0.3, -0.7, 1.1])
    lm = np.array([0.2, -0.3, 0.5]) if with_mass else None
    x0 = np.concatenate([h0, p0])

    def flow(x):
        h, p = oracle.omelyan(x[:T], x[T:], y2, r, TH, 6, 0.08, log_m=lm)
        return np.concatenate([h, p])

    J = np.zeros((2 * T, 2 * T))
    eps = 1e-6
    for j in range(2 * T):
        e = np.zeros(2 * T)
        e[j] = eps
        J[:, j] = (flow(x0 + e) - flow(x0 - e)) / (2 * eps)
    Om = np.block([[np.zeros((T, T)), np.eye(T)], [-np.eye(T), np.zeros((T, T))]])
    assert np.max(np.abs(J.T @ Om @ J - Om)) <= 1e-7
    assert abs(np.linalg.det(J) - 1.0) <= 1e-8


def _linear_gaussian(T, seed):
    """Posterior precision P and mean m of h on the linear-Gaussian target."""
    y, r, h = synth.simulate_rsv(T, TH, seed)
    z = r - TH["xi"] - TH["mu"]
    mean_a, _ = tridiag_posterior(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    Q = np.diag(np.full(T, 1 + TH["phi"] ** 2)) - TH["phi"] * (np.eye(T, k=1) + np.eye(T, k=-1))
    Q[0, 0] = Q[-1, -1] = 1.0
    P = Q / TH["sig2_eta"] + np.eye(T) / TH["sig2_u"]
    return y * y, r, h, P, mean_a + TH["mu"]


@pytest.mark.parametrize("with_mass", [False, True])
def test_converges_to_exact_flow_with_order_two(with_mass):
    T = 24
    y2, r, h0, P, m = _linear_gaussian(T, 7)
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(T)
    lm = 0.3 * rng.standard_normal(T) if with_mass else np.zeros(T)
    # exact flow of H = p^T M^-1 p / 2 + (h - m)^T P (h - m) / 2 over time 1
    G = np.block([[np.zeros((T, T)), np.diag(np.exp(-lm))], [-P, np.zeros((T, T))]])
    zt = expm(G) @ np.concatenate([h0 - m, p0])
    exact_h, exact_p = zt[:T] + m, zt[T:]
    errs, errs_lf = [], []
    dts = np.array([0.02, 0.01, 0.005])
    for dt in dts:
        k = int(round(1.0 / dt))
        h1, p1 = oracle.omelyan(h0, p0, y2, r, TH, k, dt, terms=oracle.TERM_RV,
                                log_m=lm if with_mass else None)
        errs.append(np.linalg.norm(np.concatenate([h1 - exact_h, p1 - exact_p])))
        h2, p2 = oracle.leapfrog(h0, p0, y2, r, TH, k, dt, terms=oracle.TERM_RV,
                                 log_m=lm if with_mass else None)
        errs_lf.append(np.linalg.norm(np.concatenate([h2 - exact_h, p2 - exact_p])))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 2.0) <= 0.1, (slope, errs)
    # the minimum-norm split has a smaller leading error than the leapfrog
    assert all(e < 0.5 * f for e, f in zip(errs, errs_lf)), (errs, errs_lf)


def test_energy_error_is_second_order_full_target():
    T = 1000
    y2, r, h0 = _data(T)
    p0 = np.random.default_rng(5).standard_normal(T)
    dts = np.array([0.02, 0.01, 0.005, 0.0025])
    errs = []
    for dt in dts:
        k = int(round(1.0 / dt))
        h1, p1 = oracle.omelyan(h0, p0, y2, r, TH, k, dt)
        errs.append(abs(oracle.delta_h(h0, p0, h1, p1, y2, r, TH)))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 2.0) <= 0.15, (slope, errs)


def test_trajectory_and_run_use_the_integrator():
    T = 200
    y2, r, h0 = _data(T, seed=4)
    a = oracle.trajectory(h0, y2, r, TH, 5, 0.08, seed=3, sweep=2, chain=1,
                          integrator=oracle.INT_OMELYAN)
    h1, p1 = oracle.omelyan(h0, a["p0"], y2, r, TH, 5, 0.08)
    dh = oracle.delta_h(h0, a["p0"], h1, p1, y2, r, TH)
    assert a["dH"] == dh
    b = oracle.trajectory(h0, y2, r, TH, 5, 0.08, seed=3, sweep=2, chain=1)
    assert b["dH"] != a["dH"]
    run = oracle.run(h0, TH, y2, r, 5, 0.08, 3, seed=3, first_sweep=2, chain=1,
                     update_theta=False, integrator=oracle.INT_OMELYAN)
    assert run["dH"][0] == a["dH"]


def test_linear_gaussian_posterior_matches_kalman_smoother():
    T = 50
    y, r, h_true = synth.simulate_rsv(T, TH, 31)
    z = r - TH["xi"] - TH["mu"]
    km, kv = kalman_rts(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    # k dtau = 0.24: below half a period of the stiffest mode
    out = oracle.run(h_true, TH, y * y, r, k=3, dtau=0.08, n_sweeps=100_000, seed=6,
                     update_theta=False, terms=oracle.TERM_RV, keep_h=True,
                     integrator=oracle.INT_OMELYAN)
    assert out["accepted"].mean() > 0.9
    draws = out["h_trace"][1000:]
    zm, zv = z_scores_mean_var(draws, km + TH["mu"], kv)
    assert z_rule_ok(zm), zm
    assert z_rule_ok(zv), zv
