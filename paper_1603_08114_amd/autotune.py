"""Tile-shape autotuner for the trajectory kernels.

The trajectory kernel is compiled for a few tile shapes (sites per lane S,
wavefronts per tile NW).  Which one is fastest depends on the chain lengths
(halo overhead, tail of the last round of tiles, whether chains fit one tile
and run resident), on k (halo width) and on the precision (registers per
site, hence occupancy).  ``best_shape`` times whole sweeps of the caller's
problem for every compiled shape and returns the fastest; results can be kept
in a JSON cache keyed by (precision, k, T bucket, chain-count bucket).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np
import torch

from . import api
from ._lib import RSV_F64

SHAPES = {RSV_F64: [(4, 1), (4, 2), (4, 4), (4, 8), (8, 1), (8, 2), (8, 4), (8, 8)],
          1: [(8, 1), (8, 2), (8, 4), (8, 8), (16, 1), (16, 2), (16, 4)]}


def _bucket(x):
    return 1 << max(0, math.ceil(math.log2(max(1, int(x)))))


def cache_key(precision, k, offsets, chains_per_series):
    Ts = np.diff(np.asarray(offsets))
    n_chains = (len(Ts)) * chains_per_series
    return f"p{int(precision)}|k{int(k)}|T{_bucket(Ts.max())}|c{_bucket(n_chains)}"


def time_shape(offsets, y, log_rv, h0, theta, lf, S, NW, chains_per_series=1, precision=RSV_F64,
               n_sweeps=6, update_theta=True, **kw):
    """Seconds per sweep of the problem with tile shape (S, NW)."""
    k = lf[0] if isinstance(lf, tuple) else max(a for a, _ in lf)
    smp = api.RSVSampler(offsets, y, log_rv, h0, theta, chains_per_series=chains_per_series,
                         precision=precision, max_steps=k, sites_per_lane=S, waves_per_tile=NW,
                         **kw)
    smp.sweep(0, 1, lf, update_theta=update_theta, record=())
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(smp.stream)
    smp.sweep(1, n_sweeps, lf, update_theta=update_theta, record=())
    e1.record(smp.stream)
    torch.cuda.synchronize()
    smp.close()
    return e0.elapsed_time(e1) / 1e3 / n_sweeps


def best_shape(offsets, y, log_rv, h0, theta, lf, chains_per_series=1, precision=RSV_F64,
               cache_path=None, n_sweeps=6, rounds=2, **kw):
    """(S, NW, table) for the problem; table maps "S,NW" to seconds per sweep,
    the least over `rounds` passes over the shapes (the first shape of the
    first pass also pays for the GPU's clock ramping up)."""
    k = lf[0] if isinstance(lf, tuple) else max(a for a, _ in lf)
    key = cache_key(precision, k, offsets, chains_per_series)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            S, NW = cache[key]["shape"]
            return S, NW, cache[key]["table"]
    table = {}
    for _ in range(max(1, rounds)):
        for S, NW in SHAPES[int(precision)]:
            try:
                sec = time_shape(offsets, y, log_rv, h0, theta, lf, S, NW, chains_per_series,
                                 precision, n_sweeps, **kw)
            except api.RSVError:
                continue  # shape cannot hold this k's halo
            key_s = f"{S},{NW}"
            table[key_s] = min(sec, table.get(key_s, sec))
    best = min(table, key=table.get)
    S, NW = (int(v) for v in best.split(","))
    if cache_path:
        cache[key] = {"shape": [S, NW], "table": table}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return S, NW, table
