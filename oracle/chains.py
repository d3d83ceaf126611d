"""Independent oracle chains and their per-chain posterior moments.

TEST INFRASTRUCTURE ONLY (the tests and the benchmark's cpu_baseline leg).
Each chain is the FP64 oracle sampler of this package run from the given
start; chains run one per host thread (the C oracle releases the GIL).  The
moments follow the definitions: per chain, the mean over the kept sweeps of
h_t and of h_t^2 minus the squared mean, and the same for the five theta
components.
"""
from __future__ import annotations

import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import TERMS_RSV, run


def host_threads(limit: int = 16) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def chain_moments(off, y, lr, h0s, thetas, C, k, dts, n_burn, n, seed, update_theta=True,
                  terms=TERMS_RSV, log_m=None, jitter=0.0, moves=0, seg=40, threads=None):
    """C oracle chains per series (series s: data y[off[s]:off[s+1]], start
    h0s[s] and thetas[s], step dts[s]), n_burn discarded sweeps, then n kept.
    Returns per-chain arrays h_mean, h_var (C, N: the sites of every series
    in order), theta_mean, theta_var (C, 5 S), and the wall time, the
    site-updates done and the threads used."""
    S = len(off) - 1
    threads = threads or host_threads()

    def one(job):
        s, c = job
        y2 = y[off[s]:off[s + 1]] ** 2
        r = lr[off[s]:off[s + 1]]
        kw = dict(seed=seed, chain=c, update_theta=update_theta, terms=terms, jitter=jitter,
                  moves=moves, log_m=None if log_m is None else log_m[off[s]:off[s + 1]])
        o = run(h0s[s], thetas[s], y2, r, k, dts[s], n_burn, **kw)
        h, th = o["h"], o["theta"]
        s1 = np.zeros(h.size)
        s2 = np.zeros(h.size)
        ths, done = [], 0
        while done < n:
            m = min(seg, n - done)
            o = run(h, th, y2, r, k, dts[s], m, first_sweep=n_burn + done, keep_h=True, **kw)
            s1 += o["h_trace"].sum(0)
            s2 += (o["h_trace"] ** 2).sum(0)
            ths.append(o["theta_trace"])
            h, th = o["h"], o["theta"]
            done += m
        mu = s1 / n
        tt = np.concatenate(ths)
        return mu, s2 / n - mu * mu, tt.mean(0), tt.var(0)

    jobs = [(s, c) for c in range(C) for s in range(S)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(one, jobs))
    seconds = time.perf_counter() - t0
    pick = lambda i: np.array([np.concatenate([res[c * S + s][i] for s in range(S)])
                               for c in range(C)])
    Ts = np.diff(off)
    return dict(h_mean=pick(0), h_var=pick(1), theta_mean=pick(2), theta_var=pick(3),
                seconds=seconds, site_updates=int(Ts.sum()) * C * k * (n_burn + n),
                threads=threads)
