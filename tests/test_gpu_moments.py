"""Posterior moments of GPU chains against oracle chains.

Exactness of the FP32-mixed leapfrog (precision study) and of the FP32
learned-mass path (a diagonal mass changes only the kinetic term of H,
Sec. 3, and the Metropolis test is unchanged) means their chains sample the
same posterior as FP64 oracle chains of the same sampler.  Each side runs 16 independent chains from the same
start; means and variances of every h_t and of the five theta components are
compared with standard errors from the chain-to-chain spread (Welch t).

Rule, fixed before running (paper_1603_08114_amd.diagnostics.moment_rule):
over the N sites, the fraction of p-values below 0.0027 may exceed 0.0027 by
at most three binomial standard errors, and the smallest p-value must be at
least 0.01 / N; each theta component (means and variances) needs p >=
0.01 / 5.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

from paper_1603_08114_amd import api, diagnostics as D  # noqa: E402
from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64  # noqa: E402

CHAINS = 16
KEYS = oracle.THETA_KEYS


def _cores():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 4


def gpu_moments(off, y, lr, h0s, thetas, C, k, dts, n_burn, n, precision, seed, log_mass=None,
                update_theta=True):
    """Per-chain means and variances of h_t (chains, sites of the series
    concatenated) and of theta (chains, 5) over n sweeps after n_burn."""
    S = len(off) - 1
    Ts = np.diff(off)
    h0 = np.concatenate([np.tile(h0s[s], C) for s in range(S)])
    th = [thetas[s] for s in range(S) for _ in range(C)]
    smp = api.RSVSampler(off, y, lr, h0, th, chains_per_series=C, precision=precision,
                         max_steps=k, seed=seed, log_mass=log_mass)
    lf = [(k, d) for d in dts]
    smp.sweep(0, n_burn, lf, update_theta=update_theta, record=())
    bl = 20
    out = smp.sweep(n_burn, n, lf, update_theta=update_theta, record=("theta", "accepted"),
                    batch_len=bl)
    total = out["h_batch_sum"].sum(0).cpu().numpy()
    sq = out["h_sq_sum"].cpu().numpy()
    thr = out["theta"].cpu().numpy()  # (n, chains, 5)
    acc = float(out["accepted"].float().mean())
    smp.close()
    means, variances = [], []
    for j in range(C):  # per chain: its sites of every series, in series order
        m, v = [], []
        for s in range(S):
            a = C * int(off[s]) + j * int(Ts[s])
            mu = total[a:a + Ts[s]] / n
            m.append(mu)
            v.append(sq[a:a + Ts[s]] / n - mu * mu)
        means.append(np.concatenate(m))
        variances.append(np.concatenate(v))
    th_c = thr.reshape(n, S, C, 5).transpose(2, 1, 0, 3)  # (C, S, n, 5)
    return (np.array(means), np.array(variances), th_c.mean(axis=2).reshape(C, -1),
            th_c.var(axis=2).reshape(C, -1), acc)


def oracle_moments(off, y, lr, h0s, thetas, C, k, dts, n_burn, n, seed, update_theta=True,
                   seg=40, log_m=None):
    """The same statistics from C oracle chains per series (FP64; identity
    mass unless log_m is given), one chain per host thread."""
    S = len(off) - 1

    def one(job):
        s, c = job
        y2 = y[off[s]:off[s + 1]] ** 2
        r = lr[off[s]:off[s + 1]]
        kw = dict(seed=seed, chain=c, update_theta=update_theta,
                  log_m=None if log_m is None else log_m[off[s]:off[s + 1]])
        o = oracle.run(h0s[s], thetas[s], y2, r, k, dts[s], n_burn, **kw)
        h, th = o["h"], o["theta"]
        s1 = np.zeros(h.size)
        s2 = np.zeros(h.size)
        ths, done = [], 0
        while done < n:
            m = min(seg, n - done)
            o = oracle.run(h, th, y2, r, k, dts[s], m, first_sweep=n_burn + done, keep_h=True,
                           **kw)
            s1 += o["h_trace"].sum(0)
            s2 += (o["h_trace"] ** 2).sum(0)
            ths.append(o["theta_trace"])
            h, th = o["h"], o["theta"]
            done += m
        mu = s1 / n
        tt = np.concatenate(ths)
        return mu, s2 / n - mu * mu, tt.mean(0), tt.var(0)

    jobs = [(s, c) for c in range(C) for s in range(S)]
    with ThreadPoolExecutor(_cores()) as ex:
        res = list(ex.map(one, jobs))
    means = np.array([np.concatenate([res[c * S + s][0] for s in range(S)]) for c in range(C)])
    variances = np.array([np.concatenate([res[c * S + s][1] for s in range(S)])
                          for c in range(C)])
    th_m = np.array([np.concatenate([res[c * S + s][2] for s in range(S)]) for c in range(C)])
    th_v = np.array([np.concatenate([res[c * S + s][3] for s in range(S)]) for c in range(C)])
    return means, variances, th_m, th_v


def check(gpu, ref, label, with_theta=True):
    """Apply the rule to means and variances of h and theta; print the summary."""
    report = {}
    ok_all = True
    for name, a, b in (("h_mean", gpu[0], ref[0]), ("h_var", gpu[1], ref[1])):
        z, p = D.welch_p(a, b)
        ok, summary = D.moment_rule(p)
        summary["max_abs_z"] = float(np.nanmax(np.abs(z)))
        report[name] = summary
        ok_all = ok_all and ok
    if with_theta:
        for name, a, b in (("theta_mean", gpu[2], ref[2]), ("theta_var", gpu[3], ref[3])):
            z, p = D.welch_p(a, b)
            report[name] = {"z": [round(float(v), 2) for v in z], "min_p": float(np.min(p))}
            ok_all = ok_all and bool(np.min(p) >= 0.01 / p.size)
    print(f"{label}: {report}")
    return ok_all


@pytest.mark.parametrize("precision", [RSV_F32_MIXED, RSV_F64])
def test_precision_chains_match_oracle_moments(precision):
    """The precision study at T = 2^16 (the theta of the single-series
    workloads, generator seed 2, k = 50, dtau = 0.05 (1000 / T)^(1/4), theta
    updated every sweep): 100 burn-in + 300 sweeps, FP32-mixed (and, as a
    control, FP64) GPU chains against oracle chains."""
    T, k, n_burn, n = 1 << 16, 50, 100, 300
    th = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv_long(T, th, 2)
    dt = 0.05 * (1000.0 / T) ** 0.25
    off = np.array([0, T])
    gpu = gpu_moments(off, y, lr, [h_true], [th], CHAINS, k, [dt], n_burn, n, precision, 101)
    ref = oracle_moments(off, y, lr, [h_true], [th], CHAINS, k, [dt], n_burn, n, 202)
    assert gpu[4] > 0.5
    assert check(gpu, ref, f"T=2^16 precision {precision}")


@pytest.fixture(scope="module")
def learned_mass_setup():
    """A mass network trained by the library's own kernels on plain FP64
    chains of 16 config-2-style series (seed 4), applied to 3 held-out series
    (seed 5, T ~ U{1000..4000}) at their generating theta."""
    from paper_1603_08114_amd import learned_mass as LM
    train = synth.make_batch(16, 500, 3000, seed=4)
    tr = LM.training_targets(train, C=4, k=30, warm=200, n=600)
    target = -torch.log(torch.clamp(tr["var"], min=1e-12))
    net, hist, r2 = LM.train_network(train, target, tr["theta_mean"], epochs=200)
    held = synth.make_batch(3, 1000, 4000, seed=5)
    x = net.features(held["offsets"], held["y"], held["log_rv"], synth.theta_array(held["thetas"]))
    log_m = net.log_mass(x).cpu().numpy()
    print(f"mass network: loss {hist[0]:.3f} -> {hist[-1]:.3f}, R^2 {r2:.3f}, "
          f"log m in [{log_m.min():.2f}, {log_m.max():.2f}]")
    assert np.all(np.isfinite(log_m)) and np.std(log_m) > 0.01
    return held, log_m


@pytest.mark.parametrize("update_theta", [False, True])
def test_learned_mass_fp32_chains_match_oracle_moments(learned_mass_setup, update_theta):
    """Learned-mass FP32 GPU chains against FP64 oracle chains with the same
    mass on held-out series: k = 30, dtau = 0.05 (1000 / T)^(1/4) sqrt(median
    m) (with a mass m a trajectory moves h by about dtau / sqrt(m)), 100
    burn-in + 300 sweeps from the simulated path and the generating theta;
    with theta held at its generating value (h update alone) and with theta
    updated.  Both sides run the same sampler, so a common start's transient
    is common to both; that the mass leaves the posterior unchanged is pinned
    on the oracle against the Kalman smoother of a linear-Gaussian model."""
    held, log_m = learned_mass_setup
    off = held["offsets"]
    Ts = np.diff(off)
    h0s = [held["h_true"][off[s]:off[s + 1]] for s in range(len(Ts))]
    dts = 0.05 * (1000.0 / Ts) ** 0.25 * np.array(
        [np.exp(0.5 * np.median(log_m[off[s]:off[s + 1]])) for s in range(len(Ts))])
    k, n_burn, n = 30, 100, 300
    gpu = gpu_moments(off, held["y"], held["log_rv"], h0s, held["thetas"], CHAINS, k, dts,
                      n_burn, n, RSV_F32_MIXED, 303, log_mass=log_m, update_theta=update_theta)
    ref = oracle_moments(off, held["y"], held["log_rv"], h0s, held["thetas"], CHAINS, k, dts,
                         n_burn, n, 404, update_theta=update_theta,
                         log_m=log_m.astype(np.float64))
    assert gpu[4] > 0.5
    assert check(gpu, ref, f"learned mass FP32 vs oracle, update_theta={update_theta}",
                 with_theta=update_theta)
