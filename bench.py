#!/usr/bin/env python3
"""Benchmark of the RSV HMC hot path on one MI355X.

One step = one sweep of the whole path over the single long series: momentum
refresh, k leapfrog steps, dH reduction, Metropolis test, sufficient
statistics and the theta update (rsv_hmc_sweep with n = 1 per step, the K
steps issued as one call).  Default workload: T = 2^22 sites, theta =
(0.97, -0.3, -0.2, 0.04, 0.09), k = 50, dtau tuned to ~80% acceptance,
FP64, one chain, synthetic data from the model (seed 2).

Prints ONE JSON line.  ``value`` is leapfrog site-updates per second of the
whole sweep (T * k * K / elapsed).  ``roofline`` describes the trajectory
kernel (the dominant kernel), timed with HIP events recorded by the library
on its stream around that kernel.  ``cpu_baseline`` times the FP64 CPU oracle
on a bounded sample of the same workload on the host.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "min-ESS/s and leapfrog site-updates/s; learned-mass FP32 vs plain FP64 HMC"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz, one instruction per
# lane per clock (T lane-instructions/s); FMA-counted this is the FP64 vector
# peak of 78.6 TFLOP/s, and the FP32 peak without packed FP32 (which this
# build disables; 157.3 TFLOP/s needs it)
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS_UNPACKED = 78.6
STREAM_BYTES = {"f64": 48, "f32": 24}   # read h,p,y^2,lnRV + write h,p per site-update
HOST_CORES_MAX = 16                      # the host-core share of one GPU on the measuring box


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--T", type=int, default=1 << 22)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--dtau", type=float, default=0.0, help="0 = tune to ~80%% acceptance")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--sites-per-lane", type=int, default=0,
                    help="tile shape: sites per lane (0 = the library default: 4 for f64, 8 for f32)")
    ap.add_argument("--waves-per-tile", type=int, default=0, help="0 = the library default (4)")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--level-move", type=int, default=-1, choices=[-1, 0, 1],
                    help="level move of (h, mu, xi) before each theta update; -1 = the "
                         "workload's default (off for long and small, on for batched and mass)")
    ap.add_argument("--dtau-jitter", type=float, default=-1.0,
                    help="step-size jitter j (dtau * U[1-j, 1+j] per trajectory); -1 = the "
                         "workload's default (0, the paper's fixed dtau; the batched and mass "
                         "workloads report jitter 0.5 with the level move beside their value)")
    ap.add_argument("--cpu-sweeps", type=int, default=2,
                    help="oracle sweeps timed for cpu_baseline (0 = skip)")
    ap.add_argument("--no-extras", action="store_true",
                    help="long workload only: skip the single-series and batched min-ESS/s legs")
    ap.add_argument("--workload", choices=["long", "small", "batched", "mass", "sv", "precision",
                                           "mlp"],
                    default="long",
                    help="long: one series T=2^22 (default); small: T=1000 min-ESS/s; "
                         "batched: 512 series x 4 chains, FP32-mixed; mass: learned diagonal "
                         "mass (RSV, with the SV model's arms beside); sv: the learned-mass "
                         "study on the plain SV model; precision: FP32-mixed vs FP64; mlp: the "
                         "mass network alone (BF16 MFMA)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (for counter calibration)")
    ap.add_argument("--summarize-counters", nargs=5, metavar=("FETCH", "WRITE", "CFETCH", "CWRITE",
                                                              "KEY"),
                    help="print the traffic record from four rocprofv3 counter CSVs")
    return ap.parse_args()


def tune_dtau(smp, k, T, first_sweep, target=0.8):
    """Geometric search of dtau for mean min(1, exp(-dH)) ~ target over pilot
    sweeps (theta updated, as in the measured run)."""
    import numpy as np
    dtau = 0.05 * (1000.0 / T) ** 0.25
    lo, hi = None, None
    sweep = first_sweep
    n_pilot = 60
    for _ in range(14):
        out = smp.sweep(sweep, n_pilot, (k, dtau), update_theta=True, record=("delta_h",))
        sweep += n_pilot
        dh = out["delta_h"].cpu().numpy().ravel()
        acc = float(np.mean(np.minimum(1.0, np.exp(-np.nan_to_num(dh, nan=1e9)))))
        if abs(acc - target) < 0.03:
            break
        if acc > target:
            lo = dtau
            dtau = dtau * 1.3 if hi is None else math.sqrt(dtau * hi)
        else:
            hi = dtau
            dtau = dtau / 1.3 if lo is None else math.sqrt(dtau * lo)
    return dtau, acc, sweep


def isa_figures(precision, S, NW):
    path = os.path.join(ROOT, "paper_1603_08114_amd", "isa_counts.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    return table.get(f"{precision}_S{S}_W{NW}")


KERNEL_SOURCES = ("rsv_traj.h", "rsv_traj_f64.hip", "rsv_traj_f32.hip", "rsv_device.h",
                  "rsv_exp.h", "rsv_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_traj_traffic.json")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1603_08114_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision, S, NW, T, k):
    """HBM bytes per trajectory-kernel launch from the committed counter
    summary, if it was taken on the current kernel source and this shape."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        rec = json.load(f)
    key = f"{precision}_S{S}_W{NW}_T{T}_k{k}"
    if rec.get("source_sha256") != kernel_source_hash() or key not in rec.get("launches", {}):
        return None
    return rec["launches"][key]


def summarize_counters(fetch_csv, write_csv, calib_fetch_csv, calib_write_csv, key):
    """Turn four rocprofv3 --pmc counter CSVs (k_traj FETCH_SIZE / WRITE_SIZE,
    then the same counters for the 256 MiB copy) into bytes per launch."""
    import csv

    def per_dispatch(path, counter, name_part):
        vals = {}
        for r in csv.DictReader(open(path)):
            if name_part in r["Kernel_Name"] and r["Counter_Name"] == counter:
                vals.setdefault(r["Dispatch_Id"], 0.0)
                vals[r["Dispatch_Id"]] += float(r["Counter_Value"])
        return list(vals.values())

    copy_bytes = (1 << 25) * 8
    cf = per_dispatch(calib_fetch_csv, "FETCH_SIZE", "copy")
    cw = per_dispatch(calib_write_csv, "WRITE_SIZE", "copy")
    f_scale = copy_bytes / float(np.median(cf))   # bytes per counter unit
    w_scale = copy_bytes / float(np.median(cw))
    kf = per_dispatch(fetch_csv, "FETCH_SIZE", "k_traj")
    kw = per_dispatch(write_csv, "WRITE_SIZE", "k_traj")
    rec = {"fetch_bytes": float(np.median(kf)) * f_scale,
           "write_bytes": float(np.median(kw)) * w_scale,
           "fetch_scale_bytes_per_unit": f_scale, "write_scale_bytes_per_unit": w_scale,
           "dispatches": [len(kf), len(kw)]}
    out = {"source_sha256": kernel_source_hash(), "launches": {key: rec}}
    if os.path.exists(TRAFFIC_FILE):
        old = json.load(open(TRAFFIC_FILE))
        if old.get("source_sha256") == out["source_sha256"]:
            old["launches"].update(out["launches"])
            out = old
    print(json.dumps(out, indent=1))


def host_cpu():
    """Host cores this process may use (capped at one GPU's share) and the CPU model."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return min(n, HOST_CORES_MAX), n, model


def cpu_baseline(y, lr, h0, theta, k, dtau, n_sweeps, seed, T):
    """The oracle (serial C, FP64) on the host: one chain on one core, then
    one independent chain per core on all cores (threads; the ctypes calls
    release the GIL), each chain n_sweeps sweeps of the same series."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    y2 = y * y
    t0 = time.perf_counter()
    oracle.run(h0, theta, y2, lr, k, dtau, n_sweeps, seed=seed, update_theta=True)
    dt1 = time.perf_counter() - t0
    cores, nproc, model = host_cpu()

    def one(chain):
        oracle.run(h0, theta, y2, lr, k, dtau, n_sweeps, seed=seed, chain=chain, update_theta=True)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, range(cores)))
    dtn = time.perf_counter() - t0
    return {"value": T * k * n_sweeps * cores / dtn, "unit": "site-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{cores} independent chains (one per core, threads) x {n_sweeps} sweeps "
                      f"(trajectory + theta update) of the same T={T} series, k={k}, FP64, "
                      "serial C per chain",
            "seconds": dtn, "nproc": nproc, "cpu_model": model,
            "single_core": {"value": T * k * n_sweeps / dt1, "cores": 1, "seconds": dt1}}


def min_ess_from_traces(h_trace, theta_trace):
    from paper_1603_08114_amd import diagnostics
    ess_h = diagnostics.ess_geyer(h_trace)
    ess_th = diagnostics.ess_geyer(theta_trace)
    return float(min(np.nanmin(ess_h), np.nanmin(ess_th))), ess_h, ess_th


def small_chain(jit, level, with_oracle, integrator="leapfrog"):
    """The single-series run (T = 1000, k = 20, dtau = 0.05, 500 burn-in +
    5000 sweeps, theta every sweep, FP64) on the GPU and, optionally, the same
    chain on the oracle.  The trajectory has length 1 in every case: 20
    leapfrog steps of 0.05, 10 Omelyan steps of 0.1 (20 force evaluations) or
    7 Forest-Ruth steps of 1/7 (21).  Returns (GPU record, oracle record or
    None)."""
    import torch
    import synth
    from paper_1603_08114_amd import api
    from paper_1603_08114_amd._lib import (RSV_FLAG_FOREST_RUTH, RSV_FLAG_LEVEL_MOVE,
                                           RSV_FLAG_OMELYAN)
    T, k, dtau, burn, n = 1000, 20, 0.05, 500, 5000
    iflag = 0
    if integrator == "omelyan":
        k, dtau, iflag = 10, 0.1, RSV_FLAG_OMELYAN
    elif integrator == "forest_ruth":
        k, dtau, iflag = 7, 1.0 / 7.0, RSV_FLAG_FOREST_RUTH
    theta = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv(T, theta, 1)
    flags = (RSV_FLAG_LEVEL_MOVE if level else 0) | iflag
    # the tile shape by timing sweeps of every compiled shape (one T = 1000
    # chain is latency-bound: four single-wavefront tiles without barriers
    # beat one four-wavefront tile)
    from paper_1603_08114_amd import autotune
    S_t, NW_t, _ = autotune.best_shape([0, T], y, lr, h_true, theta, (k, dtau), n_sweeps=50,
                                       seed=1, dtau_jitter=jit, flags=flags)
    smp = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=1, dtau_jitter=jit,
                         flags=flags, sites_per_lane=S_t, waves_per_tile=NW_t)
    smp.sweep(0, burn, (k, dtau), update_theta=True, record=())
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(smp.stream)
    out = smp.sweep(burn, n, (k, dtau), update_theta=True, record=("theta", "accepted"),
                    record_h=True)
    ev1.record(smp.stream)
    torch.cuda.synchronize()
    elapsed = ev0.elapsed_time(ev1) / 1e3
    min_ess, ess_h, ess_th = min_ess_from_traces(out["h"].cpu().numpy(),
                                                 out["theta"][:, 0].cpu().numpy())
    gpu = {"min_ess_per_s": min_ess / elapsed, "seconds": elapsed, "min_ess": min_ess,
           "min_ess_h": float(np.min(ess_h)),
           "min_ess_theta": dict(zip(("phi", "mu", "xi", "sig2_eta", "sig2_u"),
                                     map(float, ess_th))),
           "acceptance": float(out["accepted"].float().mean().item()),
           "site_updates_per_s": T * k * n / elapsed, "k": k, "dtau": dtau,
           "integrator": integrator, "sites_per_lane": S_t, "waves_per_tile": NW_t}
    smp.close()
    ref = None
    if with_oracle:
        import time as _t
        import oracle
        iorc = {"leapfrog": oracle.INT_LEAPFROG, "omelyan": oracle.INT_OMELYAN,
                "forest_ruth": oracle.INT_FOREST_RUTH}[integrator]
        t0 = _t.perf_counter()
        r = oracle.run(h_true, theta, y * y, lr, k, dtau, burn + n, seed=1, keep_h=True,
                       jitter=jit, moves=oracle.MOVE_LEVEL if level else 0, integrator=iorc)
        dt = _t.perf_counter() - t0
        m_ref, _, _ = min_ess_from_traces(r["h_trace"][burn:], r["theta_trace"][burn:])
        _, nproc, model = host_cpu()
        ref = {"value": m_ref / (dt * n / (burn + n)), "unit": "min-ESS/s", "cores": 1,
               "kind": "oracle", "nproc": nproc, "cpu_model": model,
               "sample": "the whole run (500 + 5000 sweeps), serial C; time pro-rated to the "
                         "5000 measured sweeps",
               "site_updates_per_s": T * k * (burn + n) / dt, "seconds": dt, "min_ess": m_ref}
    return gpu, ref


def run_small(args):
    """Single series, T = 1000, k = 20, dtau = 0.05, 500 burn-in + 5000 sweeps,
    theta every sweep, FP64: min over {h_t} and theta of the ESS per second.
    value: the paper's sampler (fixed dtau, Gibbs theta); beside it the same
    workload with step-size jitter 0.5 and the level move, with the leapfrog,
    Omelyan's and Forest-Ruth's integrators at about the same cost per
    trajectory."""
    jit = jitter_of(args, 0.0)
    level = level_of(args, False)
    gpu, ref = small_chain(jit, level, args.cpu_sweeps > 0)
    res = {"metric": METRIC, "value": gpu["min_ess_per_s"], "unit": "min-ESS/s", "n_gpus": 1,
           "steps": 5000, "warmup": 500, "ms_per_step": gpu["seconds"] / 5000 * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": "single-series RSV HMC, T=1000, k=20, dtau=0.05, FP64, "
                                  "500 burn-in + 5000 sweeps, theta every sweep"
                                  + (f", dtau jitter {jit}" if jit else "")
                                  + (", level move" if level else ""),
                      "T": 1000, "k": 20, "dtau": 0.05, "dtau_jitter": jit,
                      "level_move": bool(level), "chains": 1}}
    res.update({k_: v for k_, v in gpu.items() if k_ not in ("min_ess_per_s", "seconds")})
    if ref:
        res["cpu_baseline"] = ref
    if not jit and not level:
        g2, r2 = small_chain(0.5, True, args.cpu_sweeps > 0)
        res["with_jitter_and_level_move"] = {"gpu": g2, "oracle": r2}
        g3, r3 = small_chain(0.5, True, args.cpu_sweeps > 0, integrator="omelyan")
        res["omelyan_with_jitter_and_level_move"] = {"gpu": g3, "oracle": r3}
        g4, r4 = small_chain(0.5, True, args.cpu_sweeps > 0, integrator="forest_ruth")
        res["forest_ruth_with_jitter_and_level_move"] = {"gpu": g4, "oracle": r4}
    return res


def level_of(args, default):
    return default if args.level_move < 0 else bool(args.level_move)


def jitter_of(args, default):
    return default if args.dtau_jitter < 0 else args.dtau_jitter


def batched_data(S_=512, C_=4):
    """512 series, T ~ U{500..8000}, per-series theta (seed 3), C chains each
    starting from the simulated path."""
    import synth
    data = synth.make_batch(S_, 500, 8000, seed=3)
    off = data["offsets"]
    data["h0"] = np.concatenate([np.tile(data["h_true"][off[s]:off[s + 1]], C_)
                                 for s in range(S_)])
    data["theta0"] = [data["thetas"][s] for s in range(S_) for _ in range(C_)]
    data["C"] = C_
    return data


def batched_arm(data, k, jit, level, omelyan=False, shape=None, n=2000, bl=40,
                precision=None, terms=None, warm=500):
    """Warm-up of `warm` (500) sweeps with dtau adapted per series to acceptance 0.8
    (stochastic approximation on ln dtau, windows of 25 sweeps), then n
    measured sweeps with batch means accumulated on the device; min over
    {h_t} and theta of the ESS of each series (its chains summed), per second
    of the measured sweeps.  shape None = autotuned."""
    import torch
    from paper_1603_08114_amd import api, autotune, diagnostics, learned_mass as LM
    from paper_1603_08114_amd._lib import (RSV_F32_MIXED, RSV_FLAG_LEVEL_MOVE, RSV_FLAG_OMELYAN,
                                           RSV_TERMS_RSV)
    terms = RSV_TERMS_RSV if terms is None else terms
    precision = RSV_F32_MIXED if precision is None else precision
    off, C_ = data["offsets"], data["C"]
    Ts = np.diff(off)
    S_ = Ts.size
    k_ = k // 2 if omelyan else k
    dtau = (2.0 if omelyan else 1.0) * 0.05 * (1000.0 / Ts) ** 0.25
    kw = dict(chains_per_series=C_, precision=precision, dtau_jitter=jit, terms=terms,
              flags=(RSV_FLAG_LEVEL_MOVE if level else 0) | (RSV_FLAG_OMELYAN if omelyan else 0))
    table = None
    if shape is None:
        S_t, NW_t, table = autotune.best_shape(off, data["y"], data["log_rv"], data["h0"],
                                               data["theta0"], [(k_, d) for d in dtau],
                                               n_sweeps=4, **kw)
        print(f"[batched] autotuned tile shape S={S_t} NW={NW_t}: {table}", file=sys.stderr,
              flush=True)
    else:
        S_t, NW_t = shape
    smp = api.RSVSampler(off, data["y"], data["log_rv"], data["h0"], data["theta0"], max_steps=k_,
                         seed=3, sites_per_lane=S_t, waves_per_tile=NW_t, **kw)
    dtau, sweep, _, _ = LM.adapt(smp, k_, dtau, 0, warm, S_, C_, update_theta=True)
    lf = [(k_, d) for d in dtau]
    smp.sweep(sweep, 1, lf, update_theta=True, record=())  # apply the final decomposition
    sweep += 1
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(smp.stream)
    out = smp.sweep(sweep, n, lf, update_theta=True, record=("theta", "accepted"), batch_len=bl)
    ev1.record(smp.stream)
    torch.cuda.synchronize()
    elapsed = ev0.elapsed_time(ev1) / 1e3
    bsum = out["h_batch_sum"].cpu().numpy() / bl
    sq = out["h_sq_sum"].cpu().numpy() / n
    mean = bsum.mean(axis=0)
    var = np.maximum(sq - mean * mean, 0.0)
    ess_site = diagnostics.ess_batch_means(bsum, var, n)
    th = out["theta"].cpu().numpy()  # (n, chains, 5)
    per_series = np.empty(S_)
    for s in range(S_):
        e_h = 0.0
        e_th = np.zeros(5)
        T = int(Ts[s])
        for j in range(C_):
            c = s * C_ + j
            start = C_ * int(off[s]) + j * T
            e_h = e_h + ess_site[start:start + T]
            e_th += diagnostics.ess_geyer(th[:, c, :])
        per_series[s] = min(np.nanmin(e_h), np.nanmin(e_th))
    acc_rate = float(out["accepted"].float().mean().item())
    smp.close()
    rate = per_series / elapsed
    return dict(rate=rate, elapsed=elapsed, n=n, dtau=dtau, S=S_t, NW=NW_t, table=table,
                acceptance=acc_rate, median=float(np.median(rate)), min=float(rate.min()),
                ms_per_sweep=elapsed / n * 1e3,
                site_updates_per_s=float(Ts.sum()) * C_ * k_ * (2 if omelyan else 1) * n / elapsed)


def arm_summary(r):
    return {"median_min_ess_per_s": r["median"], "min_over_series": r["min"],
            "ms_per_step": r["ms_per_sweep"], "acceptance": r["acceptance"],
            "site_updates_per_s": r["site_updates_per_s"],
            "dtau_range": [float(r["dtau"].min()), float(r["dtau"].max())],
            "sites_per_lane": r["S"], "waves_per_tile": r["NW"]}


def run_batched(args):
    """512 series, T ~ U{500..8000}, per-series theta, 4 chains each, k = 30,
    FP32-mixed leapfrog, FP64 dH/theta; per-series dtau adapted to ~0.8
    acceptance over 500 warm-up sweeps; 2000 measured sweeps with batch means
    (50 batches of 40) accumulated on the device.  value = median over series
    of min-ESS/s under the paper's sampler (fixed dtau, Gibbs theta); beside
    it the extensions: step-size jitter 0.5 with the level move, and
    Omelyan's integrator at the same 30 force evaluations.  With --steps below
    200 (a short run for counter collection): that many measured sweeps after
    50 warm-up sweeps, the paper's sampler only, and the tile shape of
    --sites-per-lane / --waves-per-tile when given."""
    k = 30
    data = batched_data()
    Ts = np.diff(data["offsets"])
    jit = jitter_of(args, 0.0)
    level = level_of(args, False)
    if args.steps < 200:
        shape = (args.sites_per_lane, args.waves_per_tile) if args.sites_per_lane else None
        arm = batched_arm(data, k, jit, level, shape=shape, n=args.steps, bl=1, warm=50)
        return {"metric": METRIC, "value": arm["median"], "unit": "min-ESS/s (median over series)",
                "n_gpus": 1, "steps": arm["n"], "warmup": 50, "ms_per_step": arm["ms_per_sweep"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32-mixed", "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
                "config": {"workload": f"batched RSV HMC, short run of {arm['n']} sweeps (counter "
                                       "collection; ESS from so few sweeps is not meaningful)",
                           "sites_per_lane": arm["S"], "waves_per_tile": arm["NW"]},
                "site_updates_per_s": arm["site_updates_per_s"]}
    main_arm = batched_arm(data, k, jit, level)
    ext = batched_arm(data, k, 0.5, True, shape=(main_arm["S"], main_arm["NW"]))
    om = batched_arm(data, k, 0.5, True, omelyan=True)
    res = {"metric": METRIC, "value": main_arm["median"],
           "unit": "min-ESS/s (median over series)", "n_gpus": 1, "steps": main_arm["n"],
           "warmup": 500, "ms_per_step": main_arm["ms_per_sweep"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32-mixed",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": "batched RSV HMC: 512 series, T~U{500..8000}, 4 chains each, "
                                  f"k=30, FP32 leapfrog, FP64 dH/theta, 2000 sweeps"
                                  + (f", dtau jitter {jit}" if jit else "")
                                  + (", level move" if level else ""),
                      "series": int(Ts.size), "chains_per_series": 4, "k": k, "dtau_jitter": jit,
                      "level_move": bool(level), "total_sites": int(Ts.sum()),
                      "sites_per_lane": main_arm["S"], "waves_per_tile": main_arm["NW"]},
           "autotune_seconds_per_sweep": main_arm["table"],
           "min_over_series": main_arm["min"], "site_updates_per_s": main_arm["site_updates_per_s"],
           "acceptance": main_arm["acceptance"],
           "dtau_range": [float(main_arm["dtau"].min()), float(main_arm["dtau"].max())],
           "extension_jitter_0.5_level_move": arm_summary(ext),
           "extension_omelyan_k15_jitter_0.5_level_move": arm_summary(om)}
    if args.cpu_sweeps > 0:
        res["cpu_baseline"] = batched_cpu_baseline(data, k, main_arm["dtau"], jit, level)
    return res


def batched_cpu_baseline(data, k, dtau, jit, level, n_sweeps=25):
    """The oracle on all host cores, one chain per thread (OpenMP-style over
    chains): the 4 chains of the series of median length, and more series of
    similar length up to one chain per core, n_sweeps sweeps each."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    off, C_ = data["offsets"], data["C"]
    Ts = np.diff(off)
    order = np.argsort(np.abs(Ts - np.median(Ts)))
    cores, nproc, model = host_cpu()
    jobs = []
    for s in order:
        for j in range(C_):
            if len(jobs) < max(cores, C_):
                jobs.append((int(s), j))

    def one(job):
        s, j = job
        y2 = data["y"][off[s]:off[s + 1]] ** 2
        r = data["log_rv"][off[s]:off[s + 1]]
        oracle.run(data["h_true"][off[s]:off[s + 1]], data["thetas"][s], y2, r, k,
                   float(dtau[s]), n_sweeps, seed=3, chain=s * C_ + j, jitter=jit,
                   moves=oracle.MOVE_LEVEL if level else 0)

    t0 = time.perf_counter()
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(one, jobs))
    dt = time.perf_counter() - t0
    su = sum(int(Ts[s]) for s, _ in jobs) * k * n_sweeps
    return {"value": su / dt, "unit": "site-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(jobs)} chains of the series closest to the median length "
                      f"(T {int(Ts[order[0]])}..{int(max(Ts[s] for s, _ in jobs))}), "
                      f"{n_sweeps} sweeps each, one chain per thread, FP64 serial C per chain",
            "seconds": dt, "nproc": nproc, "cpu_model": model}


def mass_oracle_leg(held, net_log_m, k, n_series=8, C=16, n_burn=100, n=300, terms=None,
                    label="learned mass FP32"):
    """cpu_baseline leg of the mass workloads: C oracle chains per series on
    the host (one per thread) beside C GPU chains (learned mass, FP32-mixed),
    for the n_series held-out series closest to the median length; theta
    updated, dtau = 0.05 (1000 / T)^(1/4) sqrt(median m), 100 burn-in and
    300 kept sweeps from the simulated path and the generating theta.  The
    oracle chains are timed (the CPU baseline) and their posterior moments
    are the reference of the moment rule."""
    import oracle
    from oracle.chains import chain_moments
    from paper_1603_08114_amd import moments as M
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_TERMS_RSV
    terms = RSV_TERMS_RSV if terms is None else terms
    off = held["offsets"]
    Ts = np.diff(off)
    pick = np.sort(np.argsort(np.abs(Ts - np.median(Ts)))[:n_series])
    sub_off = np.concatenate([[0], np.cumsum(Ts[pick])])
    cat = lambda a: np.concatenate([a[off[s]:off[s + 1]] for s in pick])
    y, lr, lm = cat(held["y"]), cat(held["log_rv"]), cat(net_log_m).astype(np.float32)
    h0s = [held["h_true"][off[s]:off[s + 1]] for s in pick]
    th = [held["thetas"][s] for s in pick]
    dts = np.array([0.05 * (1000.0 / Ts[s]) ** 0.25 *
                    np.exp(0.5 * np.median(lm[sub_off[i]:sub_off[i + 1]]))
                    for i, s in enumerate(pick)])
    gpu = M.gpu_chain_moments(sub_off, y, lr, h0s, th, C, k, dts, n_burn, n, RSV_F32_MIXED, 303,
                              log_mass=lm, terms=terms)
    ref = chain_moments(sub_off, y, lr, h0s, th, C, k, dts, n_burn, n, 404,
                        terms=oracle.TERMS_RSV if terms == RSV_TERMS_RSV else terms,
                        log_m=lm.astype(np.float64))
    ok, report = M.compare(gpu, ref)
    print(f"[mass] moments {label} vs oracle: ok={ok} {report}", file=sys.stderr, flush=True)
    cores, nproc, model = host_cpu()
    baseline = {"value": ref["site_updates"] / ref["seconds"], "unit": "site-updates/s",
                "cores": ref["threads"], "kind": "oracle",
                "sample": f"{C} oracle chains x {n_series} held-out series (T {int(Ts[pick].min())}"
                          f"..{int(Ts[pick].max())}), {n_burn + n} sweeps each, learned mass, one "
                          f"chain per thread, FP64 serial C per chain",
                "seconds": ref["seconds"], "nproc": nproc, "cpu_model": model}
    moments = {"rule": "per family: fraction of p < 0.0027 <= 0.0027 + 3 binomial SE, "
                       "min p >= 0.01/N (Welch t over 16 chains per side)",
               "pass": ok, "gpu_acceptance": gpu["acceptance"], **report,
               "series": int(n_series), "chains_per_side": C, "sweeps": f"{n_burn}+{n}"}
    return baseline, moments


def mass_study(args, terms):
    """Learned diagonal mass on batched series of one model (terms): train on
    plain FP64 chains of 256 series (T ~ U{500..8000}, seed 4), evaluate on
    1024 held-out series (T ~ U{1000..16000}, seed 5), 4 chains each, k = 30,
    500 warm-up sweeps (dtau adapted per series to acceptance 0.8) and 1000
    measured sweeps per arm.  Arms under the paper's sampler (fixed dtau per
    trajectory, Gibbs theta): identity FP64, learned FP32-mixed, identity
    FP32-mixed, learned FP64; beside them the two FP32 arms with the
    extensions (step jitter 0.5 and the level move)."""
    import torch
    import synth
    from paper_1603_08114_amd import learned_mass as LM
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64, RSV_TERM_RETURN
    sv = terms == RSV_TERM_RETURN
    tag = "sv" if sv else "rsv"
    C, k = 4, 30
    n_train, n_held = (64, 128) if args.steps < 200 else (256, 1024)
    train = synth.make_batch(n_train, 500, 8000, seed=4)
    held = synth.make_batch(n_held, 1000, 16000, seed=5)
    if sv:  # the SV model has no realised-variance series: the network sees zeros there
        train["log_rv"] = np.zeros_like(train["log_rv"])
        held["log_rv"] = np.zeros_like(held["log_rv"])
    jit, level = jitter_of(args, 0.0), level_of(args, False)
    print(f"[{tag}] training targets from {n_train} series", file=sys.stderr, flush=True)
    tr = LM.training_targets(train, C=C, k=k, warm=500, n=2000, dtau_jitter=jit, level=level,
                             terms=terms)
    target = -torch.log(torch.clamp(tr["var"], min=1e-12))
    net, hist, r2 = LM.train_network(train, target, tr["theta_mean"], epochs=30)
    print(f"[{tag}] trained: loss {hist[0]:.4f} -> {hist[-1]:.4f}, R^2 {r2:.3f}",
          file=sys.stderr, flush=True)

    def arm(prec, nt, jit_, level_, seed=5):
        r = LM.run_arm(held, C, k, prec, nt, seed=seed, warm=500, n=1000, bl=25,
                       dtau_jitter=jit_, level=level_, tune_shape=True, terms=terms)
        per = np.minimum(r["ess_h"], r["ess_theta"]) / r["elapsed"]
        return r, {"median_min_ess_per_s": float(np.median(per)),
                   "min_min_ess_per_s": float(per.min()),
                   "median_ess_h_per_s": float(np.median(r["ess_h"] / r["elapsed"])),
                   "median_ess_theta_per_s": float(np.median(r["ess_theta"] / r["elapsed"])),
                   "median_ess_h_mean_per_sweep": float(np.median(r["ess_h_mean"] / r["n"])),
                   "seconds": r["elapsed"], "ms_per_sweep": r["elapsed"] / r["n"] * 1e3,
                   "acceptance": r["acceptance"],
                   "warmup_acceptance_range": [float(np.min(r["warmup_acceptance"])),
                                               float(np.max(r["warmup_acceptance"]))],
                   "median_dtau": float(np.median(r["dtau"])), "tile_shape": r["shape"],
                   "fallback_series": len(r["fallback_series"])}

    arms, runs = {}, {}
    for name, (prec, nt) in {"identity_f64": (RSV_F64, None), "learned_f32": (RSV_F32_MIXED, net),
                             "identity_f32": (RSV_F32_MIXED, None),
                             "learned_f64": (RSV_F64, net)}.items():
        runs[name], arms[name] = arm(prec, nt, jit, level)
        print(f"[{tag}] {name}: {arms[name]}", file=sys.stderr, flush=True)
    ext = {}
    for name, nt in {"identity_f32": None, "learned_f32": net}.items():
        _, ext[name] = arm(RSV_F32_MIXED, nt, 0.5, True)
        print(f"[{tag}] extension jitter 0.5 + level move, {name}: {ext[name]}", file=sys.stderr,
              flush=True)
    m = lambda a: arms[a]["median_min_ess_per_s"]
    out = {"arms_paper_sampler": arms, "arms_extension_jitter_0.5_level_move": ext,
           "gain_learned_f32_vs_identity_f64": m("learned_f32") / m("identity_f64"),
           "gain_learned_f32_vs_identity_f32": m("learned_f32") / m("identity_f32"),
           "gain_learned_f64_vs_identity_f64": m("learned_f64") / m("identity_f64"),
           "training": {"loss_first_epoch": hist[0], "loss_last_epoch": hist[-1], "r2": r2},
           "train_series": n_train, "held_out_series": n_held}
    if args.cpu_sweeps > 0:
        x = net.features(held["offsets"], held["y"], held["log_rv"],
                         synth.theta_array(held["thetas"]))
        out["cpu_baseline"], out["moments_learned_f32_vs_oracle"] = mass_oracle_leg(
            held, net.log_mass(x).cpu().numpy(), k, terms=terms,
            label=f"{tag} learned mass FP32")
    return out


def run_mass(args, terms=None):
    """Learned diagonal mass (RSV model; with terms = return only, the plain
    SV model).  value = median over series of min-ESS/s of the learned-mass
    FP32 arm under the paper's sampler; the other arms, the extension arms
    and the posterior-moment check against oracle chains beside it.  The RSV
    line also carries the SV study's arms."""
    from paper_1603_08114_amd._lib import RSV_TERM_RETURN, RSV_TERMS_RSV
    terms = RSV_TERMS_RSV if terms is None else terms
    sv = terms == RSV_TERM_RETURN
    st = mass_study(args, terms)
    a = st["arms_paper_sampler"]["learned_f32"]
    model = "SV (eq. (2) dropped)" if sv else "RSV"
    res = {"metric": METRIC, "value": a["median_min_ess_per_s"],
           "unit": "min-ESS/s (median over series)", "n_gpus": 1, "steps": 1000, "warmup": 500,
           "ms_per_step": a["ms_per_sweep"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32-mixed + bf16 network",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": f"learned diagonal mass, {model}: train {st['train_series']} "
                                  f"series, evaluate {st['held_out_series']} held-out series x 4 "
                                  "chains, k=30, paper's sampler",
                      "model": model, "train_series": st["train_series"],
                      "held_out_series": st["held_out_series"], "k": 30}}
    res.update({k_: v for k_, v in st.items() if k_ not in ("train_series", "held_out_series")})
    if not sv:
        sv_st = mass_study(args, RSV_TERM_RETURN)
        res["sv_model"] = {k_: v for k_, v in sv_st.items() if k_ != "cpu_baseline"}
    return res


MLP_FLOP_PER_SITE = 2 * (27 * 64 + 64 * 64 + 64)  # 27 -> 64 -> 64 -> 1, multiply-adds x 2
BF16_PEAK_TFLOPS = 2500.0


def run_mlp(args):
    """The learned-mass network alone: inference over the mass workload's
    1024 held-out series (T ~ U{1000..16000}, seed 5; 8.7 M sites) and one
    training epoch (batches of 8192 sites, gradient + Adam) over its 256
    training series (T ~ U{500..8000}, seed 4), BF16 on the matrix cores.
    value = inference rate in TFLOP/s at the algorithmic 11 776 FLOP per
    site (the 27 real inputs; the kernel pads them to 32)."""
    import torch
    import synth
    from paper_1603_08114_amd import mass
    held = synth.make_batch(1024, 1000, 16000, seed=5)
    train = synth.make_batch(256, 500, 8000, seed=4)
    th_h = synth.theta_array(held["thetas"])
    th_t = synth.theta_array(train["thetas"])
    mean = np.zeros(27)
    std = np.ones(27)
    net = mass.MassNet(mass.init_params(0), mean, std)
    xh = net.features(held["offsets"], held["y"], held["log_rv"], th_h)
    xt = net.features(train["offsets"], train["y"], train["log_rv"], th_t)
    tgt = torch.zeros(xt.shape[0], dtype=torch.float32, device=xt.device)
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for _ in range(2):  # warm-up
        net.forward(xh)
    net.fit(xt, tgt, 1)
    reps = max(3, min(args.steps, 20))
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(reps):
        net.features(held["offsets"], held["y"], held["log_rv"], th_h)
    ev[1].record(stream)
    for _ in range(reps):
        net.forward(xh)
    ev[2].record(stream)
    torch.cuda.synchronize()
    t_feat = ev[0].elapsed_time(ev[1]) / reps / 1e3
    t_fwd = ev[1].elapsed_time(ev[2]) / reps / 1e3
    ev[3].record(stream)
    net.fit(xt, tgt, 1)
    ev[4].record(stream)
    torch.cuda.synchronize()
    t_epoch = ev[3].elapsed_time(ev[4]) / 1e3
    n_h, n_t = int(xh.shape[0]), int(xt.shape[0])
    tf = MLP_FLOP_PER_SITE * n_h / t_fwd / 1e12
    # training: forward + backward (input and weight gradients) = 3 x the forward products
    tf_train = 3 * MLP_FLOP_PER_SITE * n_t / t_epoch / 1e12
    return {"metric": METRIC, "value": tf, "unit": "TFLOP/s (BF16 MFMA inference, 11 776 FLOP/site)",
            "n_gpus": 1, "steps": reps, "warmup": 2, "ms_per_step": t_fwd * 1e3,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
            "config": {"workload": "learned-mass network 27-64-64-1: inference over 1024 held-out "
                                   "series, one training epoch over 256 series",
                       "inference_sites": n_h, "training_sites": n_t, "batch": 8192},
            "roofline": {"bound": "mfma", "achieved": tf, "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": tf / BF16_PEAK_TFLOPS, "traffic": None},
            "inference_ms": t_fwd * 1e3, "features_ms": t_feat * 1e3,
            "inference_sites_per_s": n_h / t_fwd,
            "training_epoch_ms": t_epoch * 1e3, "training_tflops": tf_train,
            "training_sites_per_s": n_t / t_epoch}


def run_sv(args):
    """The learned-mass study on the plain SV model (the return term only):
    the identity arms are plain SV HMC under the paper's sampler."""
    from paper_1603_08114_amd._lib import RSV_TERM_RETURN
    return run_mass(args, terms=RSV_TERM_RETURN)


def run_precision(args):
    """FP32-mixed leapfrog against FP64.  (1) On T = 2^22 (theta of the
    single-series workload, seed 2, k = 50): every FP32 trajectory has an FP64
    shadow trajectory from the identical h0, momenta and ln u; value = median
    |dH_FP32 - dH_FP64|.  (2) On T = 2^16 (same theta, seed 2): 16 FP32-mixed
    and 16 FP64 GPU chains against 16 oracle chains (the cpu_baseline leg),
    100 burn-in + 300 sweeps with theta updated, posterior means and
    variances of every h_t and of theta under the moment rule."""
    import torch
    import synth
    from paper_1603_08114_amd import api
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64
    T, k = args.T, args.k
    n = max(args.steps, 50)
    theta = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv_long(T, theta, args.seed)
    s32 = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=args.seed,
                         precision=RSV_F32_MIXED)
    s64 = api.RSVSampler([0, T], y, lr, h_true.astype(np.float32).astype(np.float64), theta,
                         max_steps=k, seed=args.seed, precision=RSV_F64)
    dtau = args.dtau if args.dtau > 0 else tune_dtau(s64, k, T, 0)[0]
    lf = (k, dtau)
    s32.sweep(0, 20, lf, update_theta=True, record=())
    dA, dB, accA, accB = [], [], [], []
    for i in range(n):
        sweep = 1000 + i
        s64.h.copy_(s32.h.to(torch.float64))
        s64.theta.copy_(s32.theta)
        p0 = s64.momenta(sweep).to(torch.float32).to(torch.float64)
        lu = float(np.log(np.random.default_rng(sweep).uniform()))
        da, aa = s32.trajectory(sweep, lf, p0=p0, log_u=[lu])
        db, ab = s64.trajectory(sweep, lf, p0=p0, log_u=[lu])
        s32.theta_update(sweep, want_stats=False)
        dA.append(da.item()); dB.append(db.item()); accA.append(aa.item()); accB.append(ab.item())
    s32.close()
    s64.close()
    dA, dB = np.array(dA), np.array(dB)
    err = np.abs(dA - dB)
    res = {"metric": METRIC, "value": float(np.median(err)), "unit": "|dH_FP32 - dH_FP64| (median)",
           "n_gpus": 1, "steps": n, "warmup": 20, "ms_per_step": None, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32-mixed vs f64",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": f"precision study, T={T}, k={k}, FP32-mixed leapfrog vs FP64 "
                                  f"shadow trajectories", "T": T, "k": k, "dtau": dtau},
           "dH_abs_error": {"median": float(np.median(err)), "p99": float(np.quantile(err, 0.99)),
                            "max": float(err.max()), "median_abs_dH": float(np.median(np.abs(dB)))},
           "decision_disagreements": int(np.sum(np.array(accA) != np.array(accB))),
           "trajectories": n}
    if args.cpu_sweeps > 0:
        res["cpu_baseline"], res["moments_vs_oracle_T65536"] = precision_oracle_leg(args)
    return res


def precision_oracle_leg(args, T=1 << 16, k=50, C=16, n_burn=100, n=300):
    """cpu_baseline leg of the precision study: C oracle chains on the host
    (one per thread), timed, and C FP32-mixed and C FP64 GPU chains from the
    same start compared with them under the moment rule."""
    from oracle.chains import chain_moments
    import synth
    from paper_1603_08114_amd import moments as M
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64
    th = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv_long(T, th, args.seed)
    dt = 0.05 * (1000.0 / T) ** 0.25
    off = np.array([0, T])
    ref = chain_moments(off, y, lr, [h_true], [th], C, k, [dt], n_burn, n, 202)
    out = {"rule": "per family: fraction of p < 0.0027 <= 0.0027 + 3 binomial SE, "
                   "min p >= 0.01/N (Welch t over 16 chains per side)",
           "T": T, "k": k, "dtau": dt, "chains_per_side": C, "sweeps": f"{n_burn}+{n}"}
    for name, prec, seed in (("f32_mixed", RSV_F32_MIXED, 101), ("f64", RSV_F64, 103)):
        gpu = M.gpu_chain_moments(off, y, lr, [h_true], [th], C, k, [dt], n_burn, n, prec, seed)
        ok, report = M.compare(gpu, ref)
        print(f"[precision] moments {name} vs oracle: ok={ok} {report}", file=sys.stderr,
              flush=True)
        out[name] = {"pass": ok, "gpu_acceptance": gpu["acceptance"], **report}
    cores, nproc, model = host_cpu()
    baseline = {"value": ref["site_updates"] / ref["seconds"], "unit": "site-updates/s",
                "cores": ref["threads"], "kind": "oracle",
                "sample": f"{C} oracle chains of T={T}, k={k}, {n_burn + n} sweeps each, one "
                          f"chain per thread, FP64 serial C per chain",
                "seconds": ref["seconds"], "nproc": nproc, "cpu_model": model}
    return baseline, out


def calibrate_copy():
    """A plain device-to-device copy of 256 MiB (the FETCH_SIZE / WRITE_SIZE
    reference: each copy reads and writes exactly 256 MiB)."""
    import torch
    a = torch.empty(1 << 25, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "copy", "bytes_per_copy": a.numel() * 8, "copies": 5}))


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design in DESIGN.md, not built.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.workload != "long":
        res = {"small": run_small, "batched": run_batched, "mass": run_mass,
               "sv": run_sv, "precision": run_precision, "mlp": run_mlp}[args.workload](args)
        print(json.dumps(res), flush=True)
        return
    import numpy as np
    import torch

    import synth
    from paper_1603_08114_amd import api
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64

    T, k, K, W = args.T, args.k, args.steps, args.warmup
    theta = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv_long(T, theta, args.seed)
    prec = RSV_F64 if args.precision == "f64" else RSV_F32_MIXED
    jit = jitter_of(args, 0.0)
    smp = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=args.seed,
                         precision=prec, sites_per_lane=args.sites_per_lane,
                         waves_per_tile=args.waves_per_tile, dtau_jitter=jit)
    S = args.sites_per_lane or (4 if args.precision == "f64" else 8)
    NW = args.waves_per_tile or 4
    print(f"[bench] T={T} k={k} precision={args.precision} S={S} NW={NW}", file=sys.stderr,
          flush=True)

    sweep = 0
    if args.dtau > 0:
        dtau = args.dtau
    else:
        dtau, acc_pilot, sweep = tune_dtau(smp, k, T, sweep)
        print(f"[bench] tuned dtau={dtau:.6g} (pilot acceptance {acc_pilot:.3f})",
              file=sys.stderr, flush=True)
    lf = (k, dtau)
    tune_table = None
    if not args.sites_per_lane and not args.waves_per_tile:
        # the tile shape by timing a few sweeps of every compiled shape
        from paper_1603_08114_amd import autotune
        S_t, NW_t, tune_table = autotune.best_shape([0, T], y, lr, h_true, theta, lf,
                                                    precision=prec, n_sweeps=4,
                                                    dtau_jitter=jit, seed=args.seed)
        if (S_t, NW_t) != (S, NW):
            smp.close()
            smp = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=args.seed,
                                 precision=prec, sites_per_lane=S_t, waves_per_tile=NW_t,
                                 dtau_jitter=jit)
            S, NW = S_t, NW_t
        print(f"[bench] autotuned tile shape S={S} NW={NW}: {tune_table}", file=sys.stderr,
              flush=True)
    smp.sweep(sweep, W, lf, update_theta=True, record=())
    sweep += W
    torch.cuda.synchronize()

    api.rsv_hmc_profile(smp.ctx, K)
    stream = smp.stream
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    out = smp.sweep(sweep, K, lf, update_theta=True, record=("accepted",))
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed = ev0.elapsed_time(ev1) / 1e3
    kern_ms, n_rec = api.rsv_hmc_kernel_time(smp.ctx)
    api.rsv_hmc_profile(smp.ctx, 0)
    acc_rate = float(out["accepted"].float().mean().item())
    status, n_nonfinite = smp.check()
    assert status == 0, "non-finite state after the timed run"

    site_updates = float(T) * k * K
    value = site_updates / elapsed
    kern_avg = kern_ms / 1e3 / max(n_rec, 1)
    traj_rate = float(T) * k / kern_avg
    isa = isa_figures(args.precision, S, NW)
    # ALU roofline of the trajectory kernel: VALU lane-instructions issued per
    # second by its leapfrog loop (instructions per site-update read from the
    # gfx950 assembly x site-updates/s) against the issue peak
    roof = {"bound": "alu", "achieved": None, "peak": VALU_PEAK_T,
            "unit": "T VALU lane-instructions/s", "frac": None, "traffic": None,
            "kernel": "k_traj", "avg_launch_ms": kern_avg * 1e3, "launches": n_rec,
            "peak_is": "256 CU x 4 SIMD x 16 lanes x 2.4 GHz, one VALU instruction per lane "
                       "per clock (the nominal clock; the kernel runs near 2.07 GHz)"}
    if isa:
        roof["achieved"] = isa["valu_per_site_update"] * traj_rate / 1e12
        roof["frac"] = roof["achieved"] / VALU_PEAK_T
        roof["valu_per_site_update"] = isa["valu_per_site_update"]
        # the method's floating-point work alone (an FMA counts 2)
        flop_peak = FP64_PEAK_TFLOPS if args.precision == "f64" else FP32_PEAK_TFLOPS_UNPACKED
        flops = isa["flop_per_site_update"] * traj_rate / 1e12
        roof["flops"] = {"achieved": flops, "peak": flop_peak, "unit": "TFLOP/s",
                         "frac": flops / flop_peak,
                         "flop_per_site_update": isa["flop_per_site_update"],
                         "peak_is": ("FP64 vector" if args.precision == "f64" else
                                     "FP32 vector without packed FP32 (disabled in this build; "
                                     "157.3 TFLOP/s needs it)")}
    tr = measured_traffic(args.precision, S, NW, T, k)
    if tr:
        roof["traffic"] = tr["fetch_bytes"] + tr["write_bytes"]
        roof["traffic_detail"] = {"fetch_bytes": tr["fetch_bytes"], "write_bytes": tr["write_bytes"],
                                  "per": "k_traj launch (one trajectory)",
                                  "algorithmic_bytes": 32.0 * T}
    stream_gbs = STREAM_BYTES[args.precision] * traj_rate / 1e9

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "site-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
        "config": {"workload": f"single-series RSV HMC sweep, T={T}, k={k}, "
                               f"{args.precision.upper()}, theta updated every sweep",
                   "T": T, "k": k, "dtau": dtau, "dtau_jitter": jit, "chains": 1,
                   "sites_per_lane": S, "waves_per_tile": NW,
                   "tile_shape": "autotuned" if tune_table else "given"},
        "autotune_seconds_per_sweep": tune_table,
        "roofline": roof,
        "acceptance": acc_rate,
        "traj_kernel_site_updates_per_s": traj_rate,
        "streaming_equivalent": {"bytes_per_site_update": STREAM_BYTES[args.precision],
                                 "GB/s": stream_gbs, "frac_of_hbm_peak": stream_gbs / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    smp.close()
    if args.cpu_sweeps > 0:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(y, lr, h_true, theta, k, dtau, args.cpu_sweeps,
                                           args.seed, T)
    if not args.no_extras:
        # min-ESS/s of the paper's sampler on the single-series and batched
        # workloads, in the same run
        print("[bench] single-series min-ESS/s", file=sys.stderr, flush=True)
        g, r = small_chain(0.0, False, args.cpu_sweeps > 0)
        res["single_series_min_ess"] = {
            "workload": "one series T=1000, k=20, dtau=0.05, FP64, 500 burn-in + 5000 sweeps, "
                        "theta every sweep (the paper's sampler)",
            "min_ess_per_s": g["min_ess_per_s"], "min_ess": g["min_ess"],
            "min_ess_h": g["min_ess_h"], "min_ess_theta": g["min_ess_theta"],
            "acceptance": g["acceptance"], "ms_per_sweep": g["seconds"] / 5000 * 1e3,
            "cpu_baseline": r}
        print("[bench] batched min-ESS/s", file=sys.stderr, flush=True)
        bd = batched_data()
        b = batched_arm(bd, 30, 0.0, False, shape=(8, 1))
        res["batched_min_ess"] = {
            "workload": "512 series, T~U{500..8000}, 4 chains each, k=30, FP32 leapfrog, FP64 "
                        "dH/theta, dtau adapted to ~0.8, 2000 sweeps, 50 batch means (the "
                        "paper's sampler), tile shape 8 x 1",
            **arm_summary(b), "min_ess_per_s_median": b["median"], "min_ess_per_s_min": b["min"]}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
