"""Per-chain posterior moments of GPU chains, and the moment rule between two
sets of independent chains.

Exactness of HMC (Sec. 3: volume-preserving, reversible integrator and the
Metropolis test on H) means that any exact variant -- FP32-mixed leapfrog,
a fixed diagonal mass -- samples the same posterior as the FP64 sampler.
Two sets of C independent chains from the same start are compared through
the per-chain means and variances of every h_t and of the five theta
components, with standard errors from the chain-to-chain spread (Welch t),
by the rule of ``diagnostics.moment_rule``.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api, diagnostics as D
from ._lib import RSV_TERMS_RSV


def gpu_chain_moments(off, y, lr, h0s, thetas, C, k, dts, n_burn, n, precision, seed,
                      log_mass=None, update_theta=True, terms=RSV_TERMS_RSV, jitter=0.0,
                      flags=0, batch_len=20):
    """C chains per series on the GPU (series s starts from h0s[s] and
    thetas[s], step dts[s]); n_burn sweeps discarded, n kept, the h sums
    accumulated on the device.  Same layout of results as the oracle's
    chain_moments, plus the acceptance rate and the wall time of the kept
    sweeps."""
    S = len(off) - 1
    Ts = np.diff(off)
    h0 = np.concatenate([np.tile(h0s[s], C) for s in range(S)])
    th = [thetas[s] for s in range(S) for _ in range(C)]
    smp = api.RSVSampler(off, y, lr, h0, th, chains_per_series=C, precision=precision,
                         terms=terms, max_steps=k, seed=seed, log_mass=log_mass,
                         dtau_jitter=jitter, flags=flags)
    lf = [(k, d) for d in dts]
    smp.sweep(0, n_burn, lf, update_theta=update_theta, record=())
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(smp.stream)
    out = smp.sweep(n_burn, n, lf, update_theta=update_theta, record=("theta", "accepted"),
                    batch_len=batch_len)
    ev1.record(smp.stream)
    torch.cuda.synchronize()
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
    return dict(h_mean=np.array(means), h_var=np.array(variances),
                theta_mean=th_c.mean(axis=2).reshape(C, -1),
                theta_var=th_c.var(axis=2).reshape(C, -1), acceptance=acc,
                seconds=ev0.elapsed_time(ev1) / 1e3)


def compare(a, b, with_theta=True):
    """The moment rule between chain sets a and b (dicts as returned by
    gpu_chain_moments).  h_t means and variances: the rule over all sites;
    theta means and variances: every component p >= 0.01 / (its count).
    Returns (ok, report) with the fraction of small p-values, the smallest
    p and the largest |z| of each family."""
    report, ok_all = {}, True
    for name in ("h_mean", "h_var"):
        z, p = D.welch_p(a[name], b[name])
        ok, summary = D.moment_rule(p)
        summary["max_abs_z"] = float(np.nanmax(np.abs(z)))
        summary["ok"] = bool(ok)
        report[name] = summary
        ok_all = ok_all and ok
    if with_theta:
        for name in ("theta_mean", "theta_var"):
            z, p = D.welch_p(a[name], b[name])
            ok = bool(np.min(p) >= 0.01 / p.size)
            report[name] = {"n": int(p.size), "min_p": float(np.min(p)),
                            "min_p_limit": 0.01 / p.size,
                            "max_abs_z": float(np.max(np.abs(z))), "ok": ok}
            ok_all = ok_all and ok
    return bool(ok_all), report
