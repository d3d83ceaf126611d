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
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
STREAM_BYTES = {"f64": 48, "f32": 24}   # read h,p,y^2,lnRV + write h,p per site-update


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--T", type=int, default=1 << 22)
    ap.add_argument("--k", type=int, default=50)
    ap.add_argument("--dtau", type=float, default=0.0, help="0 = tune to ~80%% acceptance")
    ap.add_argument("--precision", choices=["f64", "f32"], default="f64")
    ap.add_argument("--sites-per-lane", type=int, default=8)
    ap.add_argument("--waves-per-tile", type=int, default=4)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--cpu-sweeps", type=int, default=2,
                    help="oracle sweeps timed for cpu_baseline (0 = skip)")
    ap.add_argument("--workload", choices=["long", "small", "batched", "mass"], default="long",
                    help="long: one series T=2^22 (default); small: T=1000 min-ESS/s; "
                         "batched: 512 series x 4 chains, FP32-mixed")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy (for counter calibration)")
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


def cpu_baseline(y, lr, h0, theta, k, dtau, n_sweeps, seed, T):
    import numpy as np
    import oracle
    t0 = time.perf_counter()
    oracle.run(h0, theta, y * y, lr, k, dtau, n_sweeps, seed=seed, update_theta=True)
    dt = time.perf_counter() - t0
    return {"value": T * k * n_sweeps / dt, "unit": "site-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_sweeps} sweeps (trajectory + theta update) of the same T={T} series, "
                      f"k={k}, FP64, serial C",
            "seconds": dt}


def min_ess_from_traces(h_trace, theta_trace):
    from paper_1603_08114_amd import diagnostics
    ess_h = diagnostics.ess_geyer(h_trace)
    ess_th = diagnostics.ess_geyer(theta_trace)
    return float(min(np.nanmin(ess_h), np.nanmin(ess_th))), ess_h, ess_th


def run_small(args):
    """Single series, T = 1000, k = 20, dtau = 0.05, 500 burn-in + 5000 sweeps,
    theta every sweep, FP64: min over {h_t} and theta of the ESS per second."""
    import torch
    import synth
    from paper_1603_08114_amd import api
    T, k, dtau, burn, n = 1000, 20, 0.05, 500, 5000
    theta = dict(synth.THETA_STAR)
    y, lr, h_true = synth.simulate_rsv(T, theta, 1)
    smp = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=1)
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
    res = {"metric": METRIC, "value": min_ess / elapsed, "unit": "min-ESS/s", "n_gpus": 1,
           "steps": n, "warmup": burn, "ms_per_step": elapsed / n * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": "single-series RSV HMC, T=1000, k=20, dtau=0.05, FP64, "
                                  "500 burn-in + 5000 sweeps, theta every sweep",
                      "T": T, "k": k, "dtau": dtau, "chains": 1},
           "site_updates_per_s": T * k * n / elapsed, "min_ess": min_ess,
           "min_ess_theta": dict(zip(("phi", "mu", "xi", "sig2_eta", "sig2_u"),
                                     map(float, ess_th))),
           "acceptance": float(out["accepted"].float().mean().item())}
    if args.cpu_sweeps > 0:
        import time as _t
        import oracle
        t0 = _t.perf_counter()
        ref = oracle.run(h_true, theta, y * y, lr, k, dtau, burn + n, seed=1, keep_h=True)
        dt = _t.perf_counter() - t0
        m_ref, _, _ = min_ess_from_traces(ref["h_trace"][burn:], ref["theta_trace"][burn:])
        res["cpu_baseline"] = {"value": m_ref / (dt * n / (burn + n)), "unit": "min-ESS/s",
                               "cores": 1, "kind": "oracle",
                               "sample": "the whole run (500 + 5000 sweeps), serial C; time "
                                         "pro-rated to the 5000 measured sweeps",
                               "site_updates_per_s": T * k * (burn + n) / dt, "seconds": dt}
    return res


def run_batched(args):
    """512 series, T ~ U{500..8000}, per-series theta, 4 chains each, k = 30,
    FP32-mixed leapfrog; per-series dtau adapted to ~0.8 acceptance over 500
    warm-up sweeps; 2000 measured sweeps with batch means (50 batches of 40)
    accumulated on the device.  value = median over series of min-ESS/s."""
    import torch
    import synth
    from paper_1603_08114_amd import api, diagnostics
    from paper_1603_08114_amd._lib import RSV_F32_MIXED
    S_, C_, k = 512, 4, 30
    data = synth.make_batch(S_, 500, 8000, seed=3)
    off = data["offsets"]
    Ts = np.diff(off)
    h0 = np.concatenate([np.tile(data["h_true"][off[s]:off[s + 1]], C_) for s in range(S_)])
    thetas = [data["thetas"][s] for s in range(S_) for _ in range(C_)]
    smp = api.RSVSampler(off, data["y"], data["log_rv"], h0, thetas, chains_per_series=C_,
                         precision=RSV_F32_MIXED, max_steps=k, seed=3)
    dtau = 0.05 * (1000.0 / Ts) ** 0.25
    sweep = 0
    for _ in range(10):  # 10 windows of 50 warm-up sweeps
        out = smp.sweep(sweep, 50, [(k, d) for d in dtau], update_theta=True,
                        record=("delta_h",))
        sweep += 50
        dh = out["delta_h"].cpu().numpy().reshape(50, S_, C_)
        acc = np.minimum(1.0, np.exp(-np.nan_to_num(dh, nan=1e9))).mean(axis=(0, 2))
        dtau = dtau * np.exp(1.5 * (acc - 0.8))
    lf = [(k, d) for d in dtau]
    smp.sweep(sweep, 1, lf, update_theta=True, record=())  # apply the final decomposition
    sweep += 1
    torch.cuda.synchronize()
    n, bl = 2000, 40
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
    rate = per_series / elapsed
    total_su = float(Ts.sum()) * C_ * k * n
    res = {"metric": METRIC, "value": float(np.median(rate)), "unit": "min-ESS/s (median over series)",
           "n_gpus": 1, "steps": n, "warmup": 500, "ms_per_step": elapsed / n * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32-mixed", "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": "batched RSV HMC: 512 series, T~U{500..8000}, 4 chains each, "
                                  "k=30, FP32 leapfrog, FP64 dH/theta, 2000 sweeps",
                      "series": S_, "chains_per_series": C_, "k": k, "total_sites": int(Ts.sum())},
           "min_over_series": float(rate.min()), "site_updates_per_s": total_su / elapsed,
           "acceptance": float(out["accepted"].float().mean().item()),
           "dtau_range": [float(dtau.min()), float(dtau.max())]}
    if args.cpu_sweeps > 0:
        import time as _t
        import oracle
        s = int(np.argsort(Ts)[S_ // 2])
        T = int(Ts[s])
        y2 = data["y"][off[s]:off[s + 1]] ** 2
        r = data["log_rv"][off[s]:off[s + 1]]
        t0 = _t.perf_counter()
        for j in range(C_):
            oracle.run(data["h_true"][off[s]:off[s + 1]], data["thetas"][s], y2, r, k,
                       float(dtau[s]), 25, seed=3, chain=s * C_ + j)
        dt = _t.perf_counter() - t0
        res["cpu_baseline"] = {"value": T * k * 25 * C_ / dt, "unit": "site-updates/s",
                               "cores": 1, "kind": "oracle",
                               "sample": f"4 chains x 25 sweeps of the median-length series "
                                         f"(T={T}), FP64 serial C", "seconds": dt}
    return res


def run_mass(args):
    """Learned diagonal mass: train on identity-FP64 chains of 256 series
    (T ~ U{500..8000}, seed 4), evaluate on 1024 held-out series
    (T ~ U{1000..16000}, seed 5), 4 chains each, k = 30, against identity
    mass, same warm-up (500 sweeps, dtau adapted per series) and 1000 measured
    sweeps per arm.  value = median over series of min-ESS/s, learned mass
    with FP32-mixed leapfrog; the other arms are reported beside it."""
    import torch
    import synth
    from paper_1603_08114_amd import learned_mass as LM
    from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64
    C, k = 4, 30
    n_train, n_held = (64, 128) if args.steps < 200 else (256, 1024)
    train = synth.make_batch(n_train, 500, 8000, seed=4)
    held = synth.make_batch(n_held, 1000, 16000, seed=5)
    print(f"[mass] training targets from {n_train} series", file=sys.stderr, flush=True)
    tr = LM.training_targets(train, C=C, k=k, warm=500, n=2000)
    target = -torch.log(torch.clamp(tr["var"], min=1e-12))
    net, hist, r2 = LM.train_network(train, target, tr["theta_mean"], epochs=30)
    print(f"[mass] trained: loss {hist[0]:.4f} -> {hist[-1]:.4f}, R^2 {r2:.3f}", file=sys.stderr,
          flush=True)
    arms = {"identity_f64": (RSV_F64, None), "learned_f32": (RSV_F32_MIXED, net),
            "identity_f32": (RSV_F32_MIXED, None), "learned_f64": (RSV_F64, net)}
    out = {}
    res_arm = {}
    for name, (prec, nt) in arms.items():
        r = LM.run_arm(held, C, k, prec, nt, seed=5, warm=500, n=1000, bl=25)
        res_arm[name] = r
        per = np.minimum(r["ess_h"], r["ess_theta"]) / r["elapsed"]
        out[name] = {"median_min_ess_per_s": float(np.median(per)),
                     "min_min_ess_per_s": float(per.min()),
                     "median_ess_h_per_s": float(np.median(r["ess_h"] / r["elapsed"])),
                     "median_ess_theta_per_s": float(np.median(r["ess_theta"] / r["elapsed"])),
                     "seconds": r["elapsed"], "acceptance": r["acceptance"],
                     "median_dtau": float(np.median(r["dtau"]))}
        print(f"[mass] {name}: {out[name]}", file=sys.stderr, flush=True)
    # posterior means of h_t and theta: learned FP32 arm vs identity FP64 arm
    a, b = res_arm["identity_f64"], res_arm["learned_f32"]
    z = ((b["mean"] - a["mean"]) / torch.sqrt(a["mcse2"] + b["mcse2"])).cpu().numpy()
    z = z[np.isfinite(z)]
    frac3 = float(np.mean(np.abs(z) > 3))
    lim = 0.0027 + 3 * np.sqrt(0.0027 * 0.9973 / z.size)
    from paper_1603_08114_amd import diagnostics
    tz = []
    S_ = len(held["offsets"]) - 1
    for r_ in (a, b):
        tr_ = r_["theta_trace"].reshape(r_["theta_trace"].shape[0], S_, C, 5)
        m = tr_.mean(axis=(0, 2))
        v = np.stack([np.stack([tr_[:, s, j, :].var(0) / diagnostics.ess_geyer(tr_[:, s, j, :])
                                for j in range(C)]).sum(0) / C ** 2 for s in range(S_)])
        tz.append((m, v))
    zt = (tz[1][0] - tz[0][0]) / np.sqrt(tz[0][1] + tz[1][1])
    gain = out["learned_f32"]["median_min_ess_per_s"] / out["identity_f64"]["median_min_ess_per_s"]
    res = {"metric": METRIC, "value": out["learned_f32"]["median_min_ess_per_s"],
           "unit": "min-ESS/s (median over series)", "n_gpus": 1, "steps": 1000, "warmup": 500,
           "ms_per_step": out["learned_f32"]["seconds"] / 1000 * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32-mixed + bf16 network",
           "data": "synthetic (RSV model eqs. (1)-(3), seeded)",
           "config": {"workload": f"learned diagonal mass: train {n_train} series, evaluate "
                                  f"{n_held} held-out series x 4 chains, k=30",
                      "train_series": n_train, "held_out_series": n_held, "k": k},
           "arms": out, "gain_learned_f32_vs_identity_f64": gain,
           "training": {"loss_first_epoch": hist[0], "loss_last_epoch": hist[-1], "r2": r2},
           "moments_learned_f32_vs_identity_f64": {
               "h_mean_frac_abs_z_gt_3": frac3, "h_frac_limit": float(lim),
               "h_max_abs_z": float(np.abs(z).max()), "n_sites": int(z.size),
               "theta_max_abs_z": float(np.nanmax(np.abs(zt))),
               "theta_frac_abs_z_gt_3": float(np.mean(np.abs(zt) > 3))}}
    return res


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
    if args.workload != "long":
        res = {"small": run_small, "batched": run_batched, "mass": run_mass}[args.workload](args)
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
    smp = api.RSVSampler([0, T], y, lr, h_true, theta, max_steps=k, seed=args.seed,
                         precision=prec, sites_per_lane=args.sites_per_lane,
                         waves_per_tile=args.waves_per_tile)
    S, NW = args.sites_per_lane, args.waves_per_tile
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
    peak = FP64_PEAK_TFLOPS if args.precision == "f64" else FP32_PEAK_TFLOPS
    roof = {"bound": "alu", "achieved": None, "peak": peak, "unit": "TFLOP/s", "frac": None,
            "traffic": None, "kernel": "k_traj", "avg_launch_ms": kern_avg * 1e3,
            "launches": n_rec}
    if isa:
        # FMA-equivalent rate of the kernel's VALU issue: 2 x (VALU instructions per
        # site-update in the leapfrog loop, from the ISA) x site-updates / s.
        per_unit = 2.0 * isa["valu_per_site_update"]
        roof["achieved"] = per_unit * traj_rate / 1e12
        roof["frac"] = roof["achieved"] / peak
        roof["flop_per_site_update"] = per_unit
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
                   "T": T, "k": k, "dtau": dtau, "chains": 1, "sites_per_lane": S,
                   "waves_per_tile": NW},
        "roofline": roof,
        "acceptance": acc_rate,
        "traj_kernel_site_updates_per_s": traj_rate,
        "streaming_equivalent": {"bytes_per_site_update": STREAM_BYTES[args.precision],
                                 "GB/s": stream_gbs, "frac_of_hbm_peak": stream_gbs / HBM_PEAK_GBS},
        "wall_s": wall,
    }
    if args.cpu_sweeps > 0:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(y, lr, h_true, theta, k, dtau, args.cpu_sweeps,
                                           args.seed, T)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
