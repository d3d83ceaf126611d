"""Pins of the oracle's leapfrog (eqs. (6)-(8)) and momentum refresh.

Properties that any correct second-order symplectic leapfrog has and that a
dropped term, wrong sign or wrong half-step would break: time reversibility,
unit Jacobian (volume preservation), energy error of order dtau^2, and
N(0, m) momenta.
"""
import numpy as np
import pytest

import oracle
import synth

TH = synth.THETA_STAR


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
    h1, p1 = oracle.leapfrog(h0, p0, y2, r, TH, 20, 0.05, log_m=lm)
    h2, p2 = oracle.leapfrog(h1, -p1, y2, r, TH, 20, 0.05, log_m=lm)
    assert np.max(np.abs(h2 - h0)) <= 1e-12 * max(1.0, np.max(np.abs(h0)))
    assert np.max(np.abs(-p2 - p0)) <= 1e-12 * max(1.0, np.max(np.abs(p0)))


def test_volume_preservation_T3():
    T = 3
    y2, r, h0 = _data(T, seed=2)
    p0 = np.array([0.3, -0.7, 1.1])
    x0 = np.concatenate([h0, p0])

    def flow(x):
        h, p = oracle.leapfrog(x[:T], x[T:], y2, r, TH, 10, 0.05)
        return np.concatenate([h, p])

    J = np.zeros((2 * T, 2 * T))
    eps = 1e-6
    for j in range(2 * T):
        e = np.zeros(2 * T)
        e[j] = eps
        J[:, j] = (flow(x0 + e) - flow(x0 - e)) / (2 * eps)
    assert abs(np.linalg.det(J) - 1.0) <= 1e-8


def test_energy_error_is_second_order():
    T = 1000
    y2, r, h0 = _data(T)
    p0 = np.random.default_rng(5).standard_normal(T)
    dts = np.array([0.02, 0.01, 0.005, 0.0025])
    errs = []
    for dt in dts:
        k = int(round(1.0 / dt))  # trajectory length l = k dtau = 1
        h1, p1 = oracle.leapfrog(h0, p0, y2, r, TH, k, dt)
        errs.append(abs(oracle.delta_h(h0, p0, h1, p1, y2, r, TH)))
    slope = np.polyfit(np.log(dts), np.log(errs), 1)[0]
    assert abs(slope - 2.0) <= 0.1, (slope, errs)


def test_single_step_order_of_operations():
    """One step from p = 0: the first half step leaves h unchanged, so the
    new p is -dtau * grad(h0) and the new h is h0 + dtau^2/2 * p."""
    T = 16
    y2, r, h0 = _data(T, seed=3)
    dt = 0.1
    h1, p1 = oracle.leapfrog(h0, np.zeros(T), y2, r, TH, 1, dt)
    g = oracle.grad(h0, y2, r, TH)
    np.testing.assert_allclose(p1, -dt * g, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(h1, h0 + 0.5 * dt * (-dt * g), rtol=1e-15, atol=1e-15)


def test_momenta_law_with_mass():
    T = 200_000
    lm = np.linspace(-2.0, 2.0, T)
    p = oracle.momenta(seed=3, sweep=1, chain=0, T=T, log_m=lm)
    z = p / np.exp(0.5 * lm)
    assert abs(z.mean()) < 4 / np.sqrt(T)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / T)
    # site t uses normal t of the momentum stream
    ref = oracle.normal_stream(3, 1, 0, oracle.TAG_MOMENTUM, 16)
    np.testing.assert_array_equal(oracle.momenta(3, 1, 0, 16), ref)


def test_trajectory_rejects_nonfinite_and_restores_state():
    T = 50
    y2, r, h0 = _data(T)
    out = oracle.trajectory(h0, y2, r, TH, k=10, dtau=50.0, seed=1)  # wildly unstable
    assert not out["accepted"]
    np.testing.assert_array_equal(out["h"], h0)


def test_trajectory_metropolis_rule():
    T = 100
    y2, r, h0 = _data(T)
    base = oracle.trajectory(h0, y2, r, TH, k=10, dtau=0.05, seed=4, sweep=2)
    dH = base["dH"]
    # accept iff log u < -dH, with the injected u on either side of the threshold
    hi = oracle.trajectory(h0, y2, r, TH, 10, 0.05, seed=4, sweep=2, log_u=-dH - 1e-9)
    lo = oracle.trajectory(h0, y2, r, TH, 10, 0.05, seed=4, sweep=2, log_u=-dH + 1e-9)
    assert hi["accepted"] and not lo["accepted"]
    tie = oracle.trajectory(h0, y2, r, TH, 10, 0.05, seed=4, sweep=2, log_u=-dH)
    assert not tie["accepted"]
    assert base["accepted"] == (oracle.log_u(4, 2, 0) < -dH)
