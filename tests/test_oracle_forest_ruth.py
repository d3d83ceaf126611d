"""Pins of the oracle's Forest-Ruth integrator (fourth order, h-first form;
Forest and Ruth 1990).

Fixed by the mathematics: on the linear-Gaussian target (eq. (1) dropped)
the exact flow is a matrix exponential of the posterior precision and the
scheme converges to it with order 4; on the full target the energy error
falls as dtau^4; the map is reversible and symplectic; the whole sampler at
fixed theta reproduces the Kalman-smoother posterior.  A wrong coefficient
(theta, 1 - 2 theta, the half drifts) drops the order to 2 or breaks
reversibility."""
import numpy as np
import pytest
from scipy.linalg import expm

import oracle
import synth
from tests._stats import z_rule_ok, z_scores_mean_var
from tests.test_oracle_omelyan import _data, _linear_gaussian
from tests.test_oracle_posterior import kalman_rts

TH = dict(synth.THETA_STAR)


def test_theta_is_the_published_root():
    th = oracle.FOREST_RUTH_THETA
    # 2 theta^3 + (1 - 2 theta)^3 = 0 removes the third-order error of the
    # symmetric composition of three leapfrogs (sizes summing to 1)
    assert abs(2 * th ** 3 + (1 - 2 * th) ** 3) < 1e-14
    assert abs(th - 1.0 / (2.0 - 2.0 ** (1.0 / 3.0))) < 1e-15


@pytest.mark.parametrize("with_mass", [False, True])
def test_converges_to_exact_flow_with_order_four(with_mass):
    T = 24
    y2, r, h0, P, m = _linear_gaussian(T, 7)
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(T)
    lm = 0.3 * rng.standard_normal(T) if with_mass else np.zeros(T)
    G = np.block([[np.zeros((T, T)), np.diag(np.exp(-lm))], [-P, np.zeros((T, T))]])
    zt = expm(G) @ np.concatenate([h0 - m, p0])
    exact = np.concatenate([zt[:T] + m, zt[T:]])
    dts = np.array([0.04, 0.02, 0.01])
    errs = []
    for dt in dts:
        k = int(round(1.0 / dt))
        h1, p1 = oracle.forest_ruth(h0, p0, y2, r, TH, k, dt, terms=oracle.TERM_RV,
                                    log_m=lm if with_mass else None)
        errs.append(np.linalg.norm(np.concatenate([h1, p1]) - exact))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 4.0) <= 0.2, (slope, errs)


def test_energy_error_is_fourth_order_full_target():
    T = 1000
    y2, r, h0 = _data(T)
    p0 = np.random.default_rng(5).standard_normal(T)
    dts = np.array([0.02, 0.01, 0.005])
    errs = []
    for dt in dts:
        k = int(round(1.0 / dt))
        h1, p1 = oracle.forest_ruth(h0, p0, y2, r, TH, k, dt)
        errs.append(abs(oracle.delta_h(h0, p0, h1, p1, y2, r, TH)))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 4.0) <= 0.3, (slope, errs)


@pytest.mark.parametrize("with_mass", [False, True])
def test_reversibility(with_mass):
    T = 1000
    y2, r, h0 = _data(T)
    rng = np.random.default_rng(0)
    p0 = rng.standard_normal(T)
    lm = 0.4 * rng.standard_normal(T) if with_mass else None
    h1, p1 = oracle.forest_ruth(h0, p0, y2, r, TH, 7, 0.05, log_m=lm)
    assert np.max(np.abs(h1 - h0)) > 1e-2
    h2, p2 = oracle.forest_ruth(h1, -p1, y2, r, TH, 7, 0.05, log_m=lm)
    assert np.max(np.abs(h2 - h0)) <= 1e-12 * max(1.0, np.max(np.abs(h0)))
    assert np.max(np.abs(-p2 - p0)) <= 1e-12 * max(1.0, np.max(np.abs(p0)))


def test_symplectic_T3():
    T = 3
    y2, r, h0 = _data(T, seed=2)
    p0 = np.array([0.3, -0.7, 1.1])
    lm = np.array([0.2, -0.3, 0.5])
    x0 = np.concatenate([h0, p0])

    def flow(x):
        h, p = oracle.forest_ruth(x[:T], x[T:], y2, r, TH, 4, 0.06, log_m=lm)
        return np.concatenate([h, p])

    J = np.zeros((2 * T, 2 * T))
    eps = 1e-6
    for j in range(2 * T):
        e = np.zeros(2 * T)
        e[j] = eps
        J[:, j] = (flow(x0 + e) - flow(x0 - e)) / (2 * eps)
    Om = np.block([[np.zeros((T, T)), np.eye(T)], [-np.eye(T), np.zeros((T, T))]])
    assert np.max(np.abs(J.T @ Om @ J - Om)) <= 1e-7


def test_trajectory_uses_the_integrator():
    T = 200
    y2, r, h0 = _data(T, seed=4)
    a = oracle.trajectory(h0, y2, r, TH, 4, 0.06, seed=3, sweep=2, chain=1,
                          integrator=oracle.INT_FOREST_RUTH)
    h1, p1 = oracle.forest_ruth(h0, a["p0"], y2, r, TH, 4, 0.06)
    assert a["dH"] == oracle.delta_h(h0, a["p0"], h1, p1, y2, r, TH)


def test_linear_gaussian_posterior_matches_kalman_smoother():
    T = 50
    y, r, h_true = synth.simulate_rsv(T, TH, 31)
    z = r - TH["xi"] - TH["mu"]
    km, kv = kalman_rts(z, TH["phi"], TH["sig2_eta"], TH["sig2_u"])
    # k dtau = 0.24: below half a period of the stiffest mode
    out = oracle.run(h_true, TH, y * y, r, k=3, dtau=0.08, n_sweeps=100_000, seed=7,
                     update_theta=False, terms=oracle.TERM_RV, keep_h=True,
                     integrator=oracle.INT_FOREST_RUTH)
    assert out["accepted"].mean() > 0.9
    draws = out["h_trace"][1000:]
    zm, zv = z_scores_mean_var(draws, km + TH["mu"], kv)
    assert z_rule_ok(zm), zm
    assert z_rule_ok(zv), zv
