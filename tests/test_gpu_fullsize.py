"""Parity at the full sizes and launch configurations the benchmark times.

* Single series T = 2^22, k = 50, FP64, tiles (4, 4) (the default) and (8, 4),
  the tuned step size: one
  trajectory on the library's own random streams against the oracle's run of
  the whole series (h' at every site rel <= 1e-12, dH abs <= 1e-9 relative to
  max(1, |dH|), the accept decision, then the theta update from the
  GPU-reduced statistics).
* The same series in FP32-mixed on injected momenta: the FP32 error bounds.
* The batched layout (512 series x 4 chains, T ~ U{500..8000}, k = 30, FP32,
  tiles (8, 1) and (8, 2), the shapes the autotuner picks there) and the held-out layout of the mass workload (1024 series x 4
  chains, T ~ U{1000..16000}, FP64, diagonal mass, tile (4, 4)): sampled
  chains (shortest, median, longest, plus a few seeded ones) against the
  oracle run on that chain alone.
* Several long FP64 chains in the split finalize (one with more slices than
  its final merge takes at once), three sweeps with the theta update, against
  the oracle run of each chain.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1603_08114_amd import api  # noqa: E402
from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64  # noqa: E402

T_LONG, K_LONG, DT_LONG = 1 << 22, 50, 0.006213052568492583


@pytest.fixture(scope="module")
def long_series():
    th = dict(synth.THETA_STAR)
    y, r, h = synth.simulate_rsv_long(T_LONG, th, 2)
    return th, y, r, h


@pytest.mark.parametrize("S,NW", [(4, 4), (8, 4)])
def test_long_series_fp64_trajectory_and_theta(long_series, S, NW):
    th, y, r, h = long_series
    smp = api.RSVSampler([0, T_LONG], y, r, h, th, max_steps=K_LONG, seed=2,
                         sites_per_lane=S, waves_per_tile=NW)
    dh, acc = smp.trajectory(7, (K_LONG, DT_LONG))
    h_gpu = smp.h.cpu().numpy()
    ref = oracle.trajectory(h, y * y, r, th, K_LONG, DT_LONG, seed=2, sweep=7, chain=0)
    dh = float(dh.item())
    assert abs(dh - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"])), (dh, ref["dH"])
    if abs(ref["dH"] + oracle.log_u(2, 7, 0)) > 1e-9:
        assert bool(acc.item()) == ref["accepted"]
        scale = max(1.0, np.max(np.abs(ref["h"])))
        assert np.max(np.abs(h_gpu - ref["h"])) <= 1e-12 * scale
        # theta from the GPU-reduced statistics of the state after the trajectory
        st = smp.theta_update(sweep=7).cpu().numpy()[0]
        ref_st = oracle.suffstats(ref["h"], r, th["mu"], th["xi"])
        np.testing.assert_allclose(st, ref_st, rtol=1e-11, atol=1e-11 * np.abs(ref_st).max())
        ref_th, _ = oracle.theta_update(T_LONG, ref_st, th, 2, 7, 0)
        got = dict(zip(oracle.THETA_KEYS, smp.theta.cpu().numpy()[0]))
        for key in oracle.THETA_KEYS:
            assert got[key] == pytest.approx(ref_th[key], rel=1e-10, abs=1e-13), key
    smp.close()


def test_long_series_fp32_error_bounds(long_series):
    th, y, r, h = long_series
    smp = api.RSVSampler([0, T_LONG], y, r, h, th, max_steps=K_LONG, seed=2,
                         precision=RSV_F32_MIXED, sites_per_lane=8, waves_per_tile=4)
    p0 = oracle.momenta(2, 3, 0, T_LONG)
    dh, acc = smp.trajectory(3, (K_LONG, DT_LONG), p0=p0, log_u=[-1e9])
    h32 = smp.h.cpu().numpy().astype(np.float64)
    h0 = h.astype(np.float32).astype(np.float64)
    p0r = p0.astype(np.float32).astype(np.float64)
    h1, p1 = oracle.leapfrog(h0, p0r, y * y, r, th, K_LONG, DT_LONG)
    ref_dh = oracle.delta_h(h0, p0r, h1, p1, y * y, r, th)
    assert np.max(np.abs(h32 - h1)) <= 2e-5
    assert abs(float(dh.item()) - ref_dh) <= 2e-3 * np.sqrt(T_LONG) / 30
    assert bool(acc.item())
    smp.close()


def _sampled(Ts, extra, seed):
    order = np.argsort(Ts)
    picks = {int(order[0]), int(order[len(Ts) // 2]), int(order[-1])}
    picks.update(int(i) for i in np.random.default_rng(seed).choice(len(Ts), extra, replace=False))
    return sorted(picks)


@pytest.mark.parametrize("NW", [1, 2])
def test_batched_layout_fp32_sampled_chains(NW):
    S_, C, k, dt = 512, 4, 30, 0.03
    data = synth.make_batch(S_, 500, 8000, seed=3)
    off = data["offsets"]
    Ts = np.diff(off)
    h0 = np.concatenate([np.tile(data["h_true"][off[s]:off[s + 1]], C) for s in range(S_)])
    ths = [data["thetas"][s] for s in range(S_) for _ in range(C)]
    smp = api.RSVSampler(off, data["y"], data["log_rv"], h0, ths, chains_per_series=C,
                         precision=RSV_F32_MIXED, max_steps=k, seed=3, sites_per_lane=8,
                         waves_per_tile=NW)
    p0 = smp.momenta(11).cpu().numpy()
    dh, acc = smp.trajectory(11, (k, dt), p0=p0, log_u=np.full(smp.n_chains, -1e9))
    h32 = smp.h.cpu().numpy().astype(np.float64)
    dh = dh.cpu().numpy()
    for s in _sampled(Ts, 3, 1):
        T = int(Ts[s])
        y2 = data["y"][off[s]:off[s + 1]] ** 2
        r = data["log_rv"][off[s]:off[s + 1]]
        for j in (0, C - 1):
            c = s * C + j
            sl = slice(C * int(off[s]) + j * T, C * int(off[s]) + (j + 1) * T)
            hh = h0[sl].astype(np.float32).astype(np.float64)
            pp = p0[sl].astype(np.float32).astype(np.float64)
            h1, p1 = oracle.leapfrog(hh, pp, y2, r, ths[c], k, dt)
            ref_dh = oracle.delta_h(hh, pp, h1, p1, y2, r, ths[c])
            assert np.max(np.abs(h32[sl] - h1)) <= 2e-5, (s, j)
            assert abs(dh[c] - ref_dh) <= 2e-3 * np.sqrt(T) / 30, (s, j)
    smp.close()


def test_mass_layout_fp64_sampled_chains():
    S_, C, k, dt = 1024, 4, 30, 0.08
    data = synth.make_batch(S_, 1000, 16000, seed=5)
    off = data["offsets"]
    Ts = np.diff(off)
    lm = np.clip(2.4 + 0.5 * np.random.default_rng(7).standard_normal(int(off[-1])), -5, 5)
    lm = lm.astype(np.float32)
    h0 = np.concatenate([np.tile(data["h_true"][off[s]:off[s + 1]], C) for s in range(S_)])
    ths = [data["thetas"][s] for s in range(S_) for _ in range(C)]
    smp = api.RSVSampler(off, data["y"], data["log_rv"], h0, ths, chains_per_series=C,
                         precision=RSV_F64, max_steps=k, seed=5, sites_per_lane=4,
                         waves_per_tile=4, log_mass=lm)
    dh, acc = smp.trajectory(2, (k, dt))
    h_gpu = smp.h.cpu().numpy()
    dh, acc = dh.cpu().numpy(), acc.cpu().numpy()
    lmd = lm.astype(np.float64)
    for s in _sampled(Ts, 3, 2):
        T = int(Ts[s])
        y2 = data["y"][off[s]:off[s + 1]] ** 2
        r = data["log_rv"][off[s]:off[s + 1]]
        for j in (0, C - 1):
            c = s * C + j
            sl = slice(C * int(off[s]) + j * T, C * int(off[s]) + (j + 1) * T)
            ref = oracle.trajectory(h0[sl], y2, r, ths[c], k, dt, seed=5, sweep=2, chain=c,
                                    log_m=lmd[off[s]:off[s + 1]])
            assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"])), (s, j)
            if abs(ref["dH"] + oracle.log_u(5, 2, c)) > 1e-9:
                assert bool(acc[c]) == ref["accepted"], (s, j)
                assert np.max(np.abs(h_gpu[sl] - ref["h"])) <= 1e-12 * max(1.0, np.abs(ref["h"]).max())
    smp.close()


def test_fp32_dh_error_has_no_coherent_bias():
    """FP32-mixed against FP64 from the same state, momenta and ln u at
    T = 2^20 (k = 50, dtau 0.05 (1000 / T)^(1/4)), after 20 sweeps from the
    simulated path: each FP32 rounding perturbs a site's contribution to dH
    independently, so |dH_FP32 - dH_FP64| grows like sqrt(T) (median 2.8e-3
    at T = 2^22 in the precision study, so ~1.4e-3 here); a coherent relative
    shift eps of every h_t would add about eps * T (1e-8 gives 1e-2 here).
    Bounds: median over 8 trajectories <= 4e-3, maximum <= 1.2e-2."""
    T, k = 1 << 20, 50
    dt = 0.05 * (1000.0 / T) ** 0.25
    th = dict(synth.THETA_STAR)
    y, r, h = synth.simulate_rsv_long(T, th, 2)
    s32 = api.RSVSampler([0, T], y, r, h, th, max_steps=k, seed=2, precision=RSV_F32_MIXED)
    s64 = api.RSVSampler([0, T], y, r, h.astype(np.float32).astype(np.float64), th,
                         max_steps=k, seed=2, precision=RSV_F64)
    s32.sweep(0, 20, (k, dt), update_theta=True, record=())
    err = []
    for i in range(8):
        sweep = 500 + i
        s64.h.copy_(s32.h.to(torch.float64))
        s64.theta.copy_(s32.theta)
        p0 = s64.momenta(sweep).to(torch.float32).to(torch.float64)
        lu = [-1e9]
        da, _ = s32.trajectory(sweep, (k, dt), p0=p0, log_u=lu)
        db, _ = s64.trajectory(sweep, (k, dt), p0=p0, log_u=lu)
        err.append(abs(float(da.item()) - float(db.item())))
    print(f"|dH_FP32 - dH_FP64| at T = 2^20: {np.round(err, 5)}")
    assert np.median(err) <= 4e-3
    assert max(err) <= 1.2e-2
    s32.close()
    s64.close()


def test_split_finalize_several_long_chains_fp64():
    """Several chains each in the split finalize (more than 128 tiles), one of
    them with more slices (34) than the final merge takes at once (32): three
    series (T = 1 000 000, 70 000, 20 000) x 2 chains, FP64, tile (4, 1), k =
    10, three sweeps with the theta update, against the oracle run of each
    chain alone (dH abs <= 1e-9 relative to max(1, |dH|), the accept
    decisions and theta after every sweep rel <= 1e-10, the final h rel <=
    1e-12; a chain stops being compared at a near-tie of its Metropolis
    test)."""
    Ts, C, k, seed, first = [1_000_000, 70_000, 20_000], 2, 10, 5, 7
    th = dict(synth.THETA_STAR)
    ys, rs, hs = [], [], []
    for i, T in enumerate(Ts):
        y, r, h = synth.simulate_rsv_long(T, th, 20 + i)
        ys.append(y); rs.append(r); hs.append(h)
    off = np.concatenate([[0], np.cumsum(Ts)])
    h0 = np.concatenate([np.tile(hs[s], C) for s in range(len(Ts))])
    dts = [0.05 * (1000.0 / T) ** 0.25 for T in Ts]
    smp = api.RSVSampler(off, np.concatenate(ys), np.concatenate(rs), h0,
                         [th] * (len(Ts) * C), chains_per_series=C, precision=RSV_F64,
                         max_steps=k, seed=seed, sites_per_lane=4, waves_per_tile=1)
    n = 3
    out = smp.sweep(first, n, [(k, d) for d in dts], record=("delta_h", "accepted", "theta"))
    dh = out["delta_h"].cpu().numpy()
    acc = out["accepted"].cpu().numpy().astype(bool)
    tht = out["theta"].cpu().numpy()
    h_gpu = smp.h.cpu().numpy()
    smp.close()
    compared = 0
    for s, T in enumerate(Ts):
        for j in range(C):
            c = s * C + j
            ref = oracle.run(hs[s], th, ys[s] ** 2, rs[s], k, dts[s], n, seed=seed, chain=c,
                             first_sweep=first)
            tie = False
            for i in range(n):
                assert abs(dh[i, c] - ref["dH"][i]) <= 1e-9 * max(1.0, abs(ref["dH"][i])), (c, i)
                if abs(ref["dH"][i] + oracle.log_u(seed, first + i, c)) <= 1e-9:
                    tie = True
                    break
                assert acc[i, c] == ref["accepted"][i], (c, i)
                np.testing.assert_allclose(tht[i, c], ref["theta_trace"][i], rtol=1e-10,
                                           atol=1e-13, err_msg=f"chain {c} sweep {i}")
                compared += 1
            if not tie:
                a = C * int(off[s]) + j * T
                scale = max(1.0, np.max(np.abs(ref["h"])))
                assert np.max(np.abs(h_gpu[a:a + T] - ref["h"])) <= 1e-12 * scale, c
    assert acc.any() and compared >= n * len(Ts) * C - 2
