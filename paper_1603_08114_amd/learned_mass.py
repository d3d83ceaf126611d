"""Learned diagonal-mass pipeline on batched series.

1. Identity-mass chains (FP64) of training series give per-site posterior
   variances; the target is -ln Var(h_t) (the log posterior precision, i.e.
   the diagonal mass that equalises the scales the leapfrog sees).
2. The network (mass.MassNet) is trained on the GPU on those targets.
3. Held-out series are sampled under four arms with the same warm-up and
   step-size adaptation: identity FP64, learned FP32-mixed, identity
   FP32-mixed, learned FP64.  The learned arms compute the mass once, after
   the first half of warm-up, from the data and the theta reached then (a
   fixed mass that depends only on data and a frozen theta keeps the
   Metropolis test exact), and adapt dtau under it for the second half.
   Identity mass is the fallback for a series whose network output is not
   finite at some site, or whose warm-up acceptance under the learned mass
   stays below 0.5 (the library itself also takes m_t = 1 at any site whose
   ln m_t is not finite).

Efficiency per series: min over {h_t} and theta of the ESS summed over the
series' chains, divided by the wall time of the measured sweeps.  ESS of h_t
comes from device-accumulated batch means, ESS of theta from Geyer's
estimator on the stored trace.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api, autotune, diagnostics, mass
from ._lib import RSV_F64, RSV_FLAG_LEVEL_MOVE, RSV_TERMS_RSV


def _series_view(off, C):
    Ts = np.diff(off)
    return Ts, np.concatenate([[0], np.cumsum(Ts * C)])


def adapt(smp, lf_k, dtau, sweep, n_sweeps, n_series, C, win=25, target=0.8, gain=2.0,
          update_theta=True):
    """Per-series dtau by stochastic approximation on ln dtau: after window i
    of `win` sweeps, ln dtau += gain / sqrt(i + 1) * (a - target), a the mean
    Metropolis probability min(1, e^-dH) over the window's trajectories of
    the series' chains.  Returns dtau, the next sweep index, the acceptance
    probability of the last window under the returned dtau's predecessor,
    and the last theta of every chain."""
    n_win = max(1, n_sweeps // win)
    for i in range(n_win):
        out = smp.sweep(sweep, win, [(lf_k, d) for d in dtau], update_theta=update_theta,
                        record=("delta_h", "theta"))
        sweep += win
        dh = out["delta_h"].cpu().numpy().reshape(win, n_series, C)
        acc = np.minimum(1.0, np.exp(-np.nan_to_num(dh, nan=1e9))).mean(axis=(0, 2))
        dtau = dtau * np.exp(gain / np.sqrt(i + 1.0) * (acc - target))
        last_theta = out["theta"].cpu().numpy()
    return dtau, sweep, acc, last_theta


def series_log_mass(log_m, off):
    """Per-series identity fallback: a series any of whose log m_t is not
    finite takes the identity mass (log m = 0) at every site.  Returns the
    array and the indices of the series that fell back."""
    lm = np.asarray(log_m, dtype=np.float32).copy()
    bad = []
    for s in range(len(off) - 1):
        seg = lm[off[s]:off[s + 1]]
        if not np.all(np.isfinite(seg)):
            seg[:] = 0.0
            bad.append(s)
    return lm, bad


def measure(smp, lf_k, dtau, sweep, n, bl, off, C, update_theta=True):
    """n measured sweeps; returns per-series min-ESS (h part, theta part),
    elapsed seconds, acceptance, and pooled per-data-site mean/var of h.
    With theta held fixed only the h part is meaningful (ess_theta is inf)."""
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(smp.stream)
    out = smp.sweep(sweep, n, [(lf_k, d) for d in dtau], update_theta=update_theta,
                    record=("theta", "accepted"), batch_len=bl)
    ev1.record(smp.stream)
    torch.cuda.synchronize()
    elapsed = ev0.elapsed_time(ev1) / 1e3
    nb = out["h_batch_sum"].shape[0]
    bm = out["h_batch_sum"] / bl
    mean = bm.mean(0)
    var = torch.clamp(out["h_sq_sum"] / (nb * bl) - mean * mean, min=0.0)
    s2 = bm.var(0, unbiased=True)
    ess = var / (s2 / nb)
    Ts, cstart = _series_view(off, C)
    th = out["theta"].cpu().numpy()
    S = len(Ts)
    ess_h = np.empty(S)
    ess_h_mean = np.empty(S)
    ess_th = np.empty(S)
    pooled_mean = torch.empty(int(off[-1]), dtype=torch.float64, device=mean.device)
    pooled_var = torch.empty_like(pooled_mean)
    for s in range(S):
        T = int(Ts[s])
        seg = slice(int(cstart[s]), int(cstart[s + 1]))
        e = ess[seg].reshape(C, T).sum(0)
        ess_h[s] = float(e.min())
        ess_h_mean[s] = float(e.mean())
        m_c = mean[seg].reshape(C, T)
        v_c = var[seg].reshape(C, T)
        pm = m_c.mean(0)
        pooled_mean[off[s]:off[s + 1]] = pm
        pooled_var[off[s]:off[s + 1]] = (v_c + m_c * m_c).mean(0) - pm * pm
        if update_theta:
            e_th = sum(diagnostics.ess_geyer(th[:, s * C + j, :]) for j in range(C))
            # components the model holds fixed (xi, sigma_u^2 without the RV
            # term) have no ESS and are left out
            ess_th[s] = float(np.nanmin(e_th))
        else:
            ess_th[s] = np.inf
    # MCSE^2 of the pooled (over chains) posterior mean of each data site
    pooled_mcse2 = torch.empty_like(pooled_mean)
    mc2 = var / ess
    for s in range(S):
        T = int(Ts[s])
        seg = slice(int(cstart[s]), int(cstart[s + 1]))
        pooled_mcse2[off[s]:off[s + 1]] = mc2[seg].reshape(C, T).sum(0) / (C * C)
    theta_mean = th.mean(axis=0).reshape(S, C, 5).mean(axis=1)
    return dict(ess_h=ess_h, ess_h_mean=ess_h_mean, ess_theta=ess_th, elapsed=elapsed, n=n,
                acceptance=float(out["accepted"].float().mean().item()),
                mean=pooled_mean, var=pooled_var, mcse2=pooled_mcse2, theta_mean=theta_mean,
                theta_trace=th)


def chains_for(data, C):
    off = data["offsets"]
    S = len(off) - 1
    h0 = np.concatenate([np.tile(data["h_true"][off[s]:off[s + 1]], C) for s in range(S)])
    thetas = [data["thetas"][s] for s in range(S) for _ in range(C)]
    return h0, thetas


def run_arm(data, C, k, precision, net=None, seed=0, warm=500, n=1000, bl=25, update_theta=True,
            dtau_jitter=0.0, level=False, tune_shape=False, log_mass=None, terms=RSV_TERMS_RSV):
    """One arm on one batch of series; returns measure() output plus dtau.
    The mass comes from `net` (evaluated after the first half of warm-up) or,
    for a reference arm, is the fixed per-site `log_mass` given.
    update_theta=False holds every chain at its series' generating theta (an
    exactness check of the h update alone: the h-conditional mixes in a few
    sweeps, so batch-means standard errors are reliable)."""
    off = data["offsets"]
    S = len(off) - 1
    Ts = np.diff(off)
    h0, thetas = chains_for(data, C)
    kw = dict(chains_per_series=C, precision=precision, max_steps=k, seed=seed, terms=terms,
              dtau_jitter=dtau_jitter, flags=RSV_FLAG_LEVEL_MOVE if level else 0)
    dtau = 0.05 * (1000.0 / Ts) ** 0.25
    shape = {}
    tkw = {k_: v for k_, v in kw.items() if k_ != "max_steps"}
    if tune_shape and net is None:
        S_, NW_, _ = autotune.best_shape(off, data["y"], data["log_rv"], h0, thetas,
                                         [(k, d) for d in dtau], n_sweeps=4, **tkw)
        shape = dict(sites_per_lane=S_, waves_per_tile=NW_)
    smp = api.RSVSampler(off, data["y"], data["log_rv"], h0, thetas, **kw, **shape)
    dtau, sweep, _, theta_now = adapt(smp, k, dtau, 0, warm // 2, S, C,
                                      update_theta=update_theta)
    lm_host, fallback = None, []
    learned = net is not None or log_mass is not None
    if learned:
        if net is not None:
            theta_hat = theta_now.mean(axis=0).reshape(S, C, 5).mean(axis=1)
            x = net.features(off, data["y"], data["log_rv"], theta_hat)
            lm_host, fallback = series_log_mass(net.log_mass(x).cpu().numpy(), off)
        else:
            lm_host, fallback = series_log_mass(log_mass, off)
        state = smp.h.to(torch.float64).cpu().numpy()
        th_now = smp.theta.cpu().numpy()
        smp.close()
        # a mass m moves h by about dtau / sqrt(m) per step: start the second
        # half of warm-up from dtau sqrt(median m) of each series
        dtau = dtau * np.array([np.exp(0.5 * np.median(lm_host[off[s]:off[s + 1]]))
                                for s in range(S)])
        if tune_shape:
            S_, NW_, _ = autotune.best_shape(off, data["y"], data["log_rv"], state, th_now,
                                             [(k, d) for d in dtau], n_sweeps=4,
                                             log_mass=lm_host, **tkw)
            shape = dict(sites_per_lane=S_, waves_per_tile=NW_)
        smp = api.RSVSampler(off, data["y"], data["log_rv"], state, th_now,
                             log_mass=lm_host, **kw, **shape)
    dtau, sweep, acc, _ = adapt(smp, k, dtau, sweep, warm // 2, S, C, update_theta=update_theta)
    if learned and np.any(acc < 0.5):
        # identity fallback for the series whose warm-up acceptance under the
        # learned mass stayed below 0.5: they restart the second half of
        # warm-up with m = 1 from their state at this point
        low = np.flatnonzero(acc < 0.5)
        for s in low:
            dtau[s] = dtau[s] / np.exp(0.5 * np.median(lm_host[off[s]:off[s + 1]]))
            lm_host[off[s]:off[s + 1]] = 0.0
        fallback = sorted(set(fallback) | set(int(s) for s in low))
        state = smp.h.to(torch.float64).cpu().numpy()
        th_now = smp.theta.cpu().numpy()
        smp.close()
        smp = api.RSVSampler(off, data["y"], data["log_rv"], state, th_now,
                             log_mass=lm_host, **kw, **shape)
        dtau, sweep, acc, _ = adapt(smp, k, dtau, sweep, warm // 2, S, C,
                                    update_theta=update_theta)
    res = measure(smp, k, dtau, sweep, n, bl, off, C, update_theta=update_theta)
    res["dtau"] = dtau
    res["warmup_acceptance"] = acc
    res["log_mass"] = lm_host
    res["fallback_series"] = fallback
    res["shape"] = shape
    smp.close()
    return res


def training_targets(data, C=4, k=30, warm=500, n=2000, seed=0, dtau_jitter=0.0, level=False,
                     terms=RSV_TERMS_RSV):
    """Pooled per-site posterior mean and variance from identity FP64 chains."""
    res = run_arm(data, C, k, RSV_F64, None, seed=seed, warm=warm, n=n, bl=40,
                  dtau_jitter=dtau_jitter, level=level, terms=terms)
    return res


def feature_stats(data, theta_series):
    """Mean and standard deviation of the 27 raw inputs over all sites."""
    off = data["offsets"]
    ly = np.log(data["y"] ** 2 + 1e-8)
    lr = data["log_rv"]
    mean = np.empty(27)
    std = np.empty(27)
    mean[:11] = ly.mean()
    std[:11] = ly.std()
    mean[11:22] = lr.mean()
    std[11:22] = lr.std()
    th = np.asarray(theta_series).reshape(-1, 5)
    Ts = np.diff(off)
    w = Ts / Ts.sum()
    mt = (th * w[:, None]).sum(0)
    mean[22:] = mt
    std[22:] = np.sqrt(((th - mt) ** 2 * w[:, None]).sum(0)) + 1e-12
    # an input that is constant over the training set (the realised-variance
    # window of the SV model) is centred and left unscaled
    std[std == 0.0] = 1.0
    return mean, std


def train_network(data, targets, theta_series, epochs=30, batch=8192, lr=2e-3, seed=0):
    mean, std = feature_stats(data, theta_series)
    net = mass.MassNet(mass.init_params(seed), mean, std)
    x = net.features(data["offsets"], data["y"], data["log_rv"], theta_series)
    tgt = targets.to(torch.float32).contiguous()
    hist = net.fit(x, tgt, epochs, batch=batch, lr=lr, seed=seed)
    pred = net.forward(x)
    r2 = 1.0 - float(((pred - tgt) ** 2).mean() / tgt.var())
    return net, hist, r2
