"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Same seeded synthetic inputs on both sides; momenta and Metropolis uniforms
either injected or drawn by both sides' independent Philox4x64-10 streams.
Bars: h after one trajectory rel <= 1e-12 (FP64), dH abs <= 1e-9, identical
accept decisions except near-ties |dH + ln u| < 1e-9, theta rel <= 1e-10,
sufficient statistics rel <= 1e-12.
"""
import numpy as np
import pytest

import oracle
import synth
from _parity import NEAR_TIE, sweeps_with_resync

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1603_08114_amd import api  # noqa: E402
from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64, RSV_TERM_RV  # noqa: E402

TH = dict(synth.THETA_STAR)


def make_series(Ts, seed, thetas=None):
    ys, rs, hs = [], [], []
    for i, T in enumerate(Ts):
        th = TH if thetas is None else thetas[i]
        y, r, h = synth.simulate_rsv_long(T, th, seed + 17 * i)
        ys.append(y); rs.append(r); hs.append(h)
    offsets = np.concatenate([[0], np.cumsum(Ts)]).astype(np.int64)
    return offsets, ys, rs, hs


def state_from(hs, C, jitter=0.0, seed=0):
    rng = np.random.default_rng(seed)
    parts = []
    for h in hs:
        for j in range(C):
            parts.append(h + jitter * j * rng.standard_normal(h.size))
    return np.concatenate(parts)


def sampler(Ts, C=1, seed=5, k=20, precision=RSV_F64, thetas=None, log_mass=None, S=0,
            terms=3, jitter=0.05, NW=0, dtau_jitter=0.0, flags=0):
    offsets, ys, rs, hs = make_series(Ts, 100 + seed, thetas)
    h0 = state_from(hs, C, jitter)
    th = [thetas[s] if thetas else TH for s in range(len(Ts)) for _ in range(C)]
    smp = api.RSVSampler(offsets, np.concatenate(ys), np.concatenate(rs), h0, th,
                         chains_per_series=C, precision=precision, max_steps=k, seed=seed,
                         log_mass=log_mass, sites_per_lane=S, waves_per_tile=NW, terms=terms,
                         dtau_jitter=dtau_jitter, flags=flags)
    return smp, offsets, ys, rs, h0, th


def chain_slices(offsets, C):
    out = []
    for s in range(offsets.size - 1):
        T = int(offsets[s + 1] - offsets[s])
        for j in range(C):
            start = C * int(offsets[s]) + j * T
            out.append((s, slice(start, start + T)))
    return out


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


SHAPES = [
    ([1000], 1, 20, 0.05),          # single-series workload, one tile
    ([3], 1, 20, 0.05),             # minimum length
    ([512], 1, 20, 0.05),           # exactly 64 * sites-per-lane
    ([513, 4000], 2, 30, 0.04),     # ragged, several tiles, two chains per series
    ([9001], 1, 50, 0.02),          # many tiles with k = 50 halos
]


@pytest.mark.parametrize("Ts,C,k,dt", SHAPES)
@pytest.mark.parametrize("S,NW", [(4, 1), (8, 1), (4, 2), (4, 4), (4, 8), (8, 2), (8, 4), (8, 8)])
def test_trajectory_injected_momenta_f64(Ts, C, k, dt, S, NW):
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k, S=S, NW=NW)
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(h0.size)
    log_u = np.log(rng.uniform(size=smp.n_chains))
    dh, acc = smp.trajectory(7, (k, dt), p0=p0, log_u=log_u)
    h_gpu = smp.h.cpu().numpy()
    dh, acc = dh.cpu().numpy(), acc.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        y2, r = ys[s] ** 2, rs[s]
        h1, p1 = oracle.leapfrog(h0[sl], p0[sl], y2, r, th[c], k, dt)
        dH = oracle.delta_h(h0[sl], p0[sl], h1, p1, y2, r, th[c])
        assert abs(dh[c] - dH) <= 1e-9 * max(1.0, abs(dH)), (c, dh[c], dH)
        ref = oracle.trajectory(h0[sl], y2, r, th[c], k, dt, p0=p0[sl], log_u=log_u[c])
        if abs(dH + log_u[c]) > NEAR_TIE:
            assert bool(acc[c]) == ref["accepted"]
            expect = h1 if ref["accepted"] else h0[sl]
            assert rel_inf(h_gpu[sl], expect) <= 1e-12, (c, rel_inf(h_gpu[sl], expect))


@pytest.mark.parametrize("Ts,C", [([1000], 1), ([700, 3000, 64], 3)])
def test_momenta_match_oracle_streams(Ts, C):
    smp, offsets, ys, rs, h0, th = sampler(Ts, C)
    p = smp.momenta(11).cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        ref = oracle.momenta(smp.pb.seed, 11, c, sl.stop - sl.start)
        np.testing.assert_allclose(p[sl], ref, rtol=1e-14, atol=1e-14)


def test_momenta_with_mass():
    T = 777
    lm = (0.4 * np.random.default_rng(1).standard_normal(T)).astype(np.float32)
    smp, offsets, ys, rs, h0, th = sampler([T], 1, log_mass=lm)
    p = smp.momenta(4).cpu().numpy()
    ref = oracle.momenta(smp.pb.seed, 4, 0, T, log_m=lm.astype(np.float64))
    np.testing.assert_allclose(p, ref, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("mass", [False, True])
def test_f32_momenta_are_the_streams_in_fp32(mass):
    """On the FP32-mixed path the momenta take eight sites per Philox block
    and an FP32 Box-Muller: rsv_hmc_momenta returns FP32 values that agree
    with the oracle's FP64 evaluation of that layout (times sqrt(m_t)) to a
    few FP32 ulps, and a trajectory on the context's own streams equals, bit
    for bit, the one from those momenta injected (the kernel draws exactly
    these)."""
    Ts, C, k, dt = [700, 3000, 64], 2, 20, 0.05
    n = int(np.sum(Ts))
    lm = (0.4 * np.sin(np.arange(n) * 0.03)).astype(np.float32) if mass else None

    def make():
        return sampler(Ts, C, k=k, precision=RSV_F32_MIXED, log_mass=lm)

    smp, offsets, ys, rs, h0, th = make()
    p = smp.momenta(11).cpu().numpy()
    np.testing.assert_array_equal(p.astype(np.float32).astype(np.float64), p)
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        T = sl.stop - sl.start
        lms = None if lm is None else lm[offsets[s]:offsets[s + 1]].astype(np.float64)
        ref = oracle.momenta_f32(smp.pb.seed, 11, c, T, log_m=lms)
        np.testing.assert_allclose(p[sl], ref, rtol=4e-6, atol=4e-6)
    log_u = np.log(np.random.default_rng(3).uniform(size=smp.n_chains))
    dh_a, acc_a = smp.trajectory(11, (k, dt), log_u=log_u)
    h_a = smp.h.clone()
    smp.close()
    smp, *_ = make()
    dh_b, acc_b = smp.trajectory(11, (k, dt), p0=p, log_u=log_u)
    assert torch.equal(h_a, smp.h)
    assert torch.equal(dh_a, dh_b)
    assert torch.equal(acc_a, acc_b)
    assert bool(acc_a.any())
    smp.close()


@pytest.mark.parametrize("Ts,C,k,dt", SHAPES[:4])
def test_trajectory_own_streams_f64(Ts, C, k, dt):
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k)
    dh, acc = smp.trajectory(3, (k, dt))
    h_gpu = smp.h.cpu().numpy()
    dh, acc = dh.cpu().numpy(), acc.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        ref = oracle.trajectory(h0[sl], ys[s] ** 2, rs[s], th[c], k, dt, seed=smp.pb.seed,
                                sweep=3, chain=c)
        assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
        if abs(ref["dH"] + oracle.log_u(smp.pb.seed, 3, c)) > NEAR_TIE:
            assert bool(acc[c]) == ref["accepted"]
            assert rel_inf(h_gpu[sl], ref["h"]) <= 1e-12


def test_trajectory_with_mass_f64():
    Ts, k, dt = [1500, 600], 20, 0.04
    lm = (0.3 * np.random.default_rng(9).standard_normal(sum(Ts))).astype(np.float32)
    smp, offsets, ys, rs, h0, th = sampler(Ts, 1, k=k, log_mass=lm)
    dh, acc = smp.trajectory(2, (k, dt))
    h_gpu, dh, acc = smp.h.cpu().numpy(), dh.cpu().numpy(), acc.cpu().numpy()
    lmd = lm.astype(np.float64)
    for c, (s, sl) in enumerate(chain_slices(offsets, 1)):
        dsl = slice(int(offsets[s]), int(offsets[s + 1]))
        ref = oracle.trajectory(h0[sl], ys[s] ** 2, rs[s], th[c], k, dt, seed=smp.pb.seed,
                                sweep=2, chain=c, log_m=lmd[dsl])
        assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
        assert bool(acc[c]) == ref["accepted"]
        assert rel_inf(h_gpu[sl], ref["h"]) <= 1e-12


def test_trajectory_with_mass_multi_tile_chains_f64():
    """Learned-mass scale (log m ~ 2.4 +- 0.7) on chains that span several
    tiles, with several chains per series sharing the series' mass."""
    Ts, C, k, dt = [5000, 1300], 2, 30, 0.08
    lm = np.clip(2.4 + 0.7 * np.random.default_rng(4).standard_normal(sum(Ts)), -5, 5)
    lm = lm.astype(np.float32)
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k, log_mass=lm)
    dh, acc = smp.trajectory(6, (k, dt))
    h_gpu, dh, acc = smp.h.cpu().numpy(), dh.cpu().numpy(), acc.cpu().numpy()
    lmd = lm.astype(np.float64)
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        dsl = slice(int(offsets[s]), int(offsets[s + 1]))
        ref = oracle.trajectory(h0[sl], ys[s] ** 2, rs[s], th[c], k, dt, seed=smp.pb.seed,
                                sweep=6, chain=c, log_m=lmd[dsl])
        assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
        if abs(ref["dH"] + oracle.log_u(smp.pb.seed, 6, c)) > NEAR_TIE:
            assert bool(acc[c]) == ref["accepted"]
            assert rel_inf(h_gpu[sl], ref["h"]) <= 1e-12


def test_f32_mixed_trajectory_with_mass_error_vs_f64():
    """FP32 leapfrog with a diagonal mass against the FP64 oracle on the same
    (FP32-rounded) momenta and mass; bounds as for the identity-mass case."""
    Ts, C, k, dt = [3000, 700], 2, 30, 0.08
    lm = np.clip(2.4 + 0.7 * np.random.default_rng(5).standard_normal(sum(Ts)), -5, 5)
    lm = lm.astype(np.float32)
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k, precision=RSV_F32_MIXED, log_mass=lm)
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(smp.n_state) * np.exp(0.5 * np.concatenate(
        [np.tile(lm[offsets[s]:offsets[s + 1]], C) for s in range(len(Ts))]))
    dh, acc = smp.trajectory(1, (k, dt), p0=p0, log_u=np.full(smp.n_chains, -50.0))
    h32 = smp.h.cpu().numpy().astype(np.float64)
    h0_32 = h0.astype(np.float32).astype(np.float64)
    lmd = lm.astype(np.float64)
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        dsl = slice(int(offsets[s]), int(offsets[s + 1]))
        p0c = p0[sl].astype(np.float32).astype(np.float64)
        h1, p1 = oracle.leapfrog(h0_32[sl], p0c, ys[s] ** 2, rs[s], th[c], k, dt,
                                 log_m=lmd[dsl])
        dH = oracle.delta_h(h0_32[sl], p0c, h1, p1, ys[s] ** 2, rs[s], th[c], log_m=lmd[dsl])
        assert np.max(np.abs(h32[sl] - h1)) <= 2e-5
        assert abs(dh[c].item() - dH) <= 2e-3 * np.sqrt(sl.stop - sl.start) / 30
    assert bool(acc.all())


@pytest.mark.parametrize("Ts,C", [([1000], 1), ([513, 4000], 2)])
def test_trajectory_with_step_jitter_f64(Ts, C):
    k, dt, j = 20, 0.05, 0.4
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k, dtau_jitter=j)
    dh, acc = smp.trajectory(12, (k, dt))
    h_gpu, dh, acc = smp.h.cpu().numpy(), dh.cpu().numpy(), acc.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        ref = oracle.trajectory(h0[sl], ys[s] ** 2, rs[s], th[c], k, dt, seed=smp.pb.seed,
                                sweep=12, chain=c, jitter=j)
        assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
        if abs(ref["dH"] + oracle.log_u(smp.pb.seed, 12, c)) > NEAR_TIE:
            assert bool(acc[c]) == ref["accepted"]
            assert rel_inf(h_gpu[sl], ref["h"]) <= 1e-12


def test_sweep_with_step_jitter_matches_oracle():
    Ts, C, k, dt, n, j = [600, 2500], 2, 30, 0.04, 40, 0.3
    sweep_parity(Ts, C, k, dt, n, 50, thetas=synth.draw_batch_thetas(len(Ts), 6), jitter=j)


@pytest.mark.parametrize("terms", [3, 1, 2])
def test_sweep_with_level_move_matches_oracle(terms):
    """Level move before every theta update (ragged chains over several tiles,
    two chains per series, jittered step): accept sequence, dH, theta and h of
    every sweep against the oracle's chain with the same move."""
    from paper_1603_08114_amd._lib import RSV_FLAG_LEVEL_MOVE
    Ts, C, k, dt, n, j = [700, 2600], 2, 20, 0.04, 40, 0.3
    refs = sweep_parity(Ts, C, k, dt, n, 30, thetas=synth.draw_batch_thetas(len(Ts), 8),
                        jitter=j, moves=oracle.MOVE_LEVEL, terms=terms,
                        flags=RSV_FLAG_LEVEL_MOVE)
    for ref in refs:  # the move did move the level: mu changes on (almost) every sweep
        assert np.mean(np.diff(ref["theta_trace"][:, 1]) != 0) > 0.9


def test_sv_model_sweeps_match_oracle():
    """The plain SV model (eq. (2) dropped: the return term only) under the
    paper's sampler -- fixed dtau, no level move -- on ragged series over
    several tiles, two chains each: accept sequence, dH, theta and h of every
    sweep against the oracle's chain; xi and sigma_u^2 stay at their start."""
    Ts, C, k, dt, n = [700, 2600], 2, 20, 0.04, 40
    refs = sweep_parity(Ts, C, k, dt, n, 30, thetas=synth.draw_batch_thetas(len(Ts), 12),
                        terms=1)
    for ref in refs:
        tr = ref["theta_trace"]
        assert np.all(tr[:, 2] == tr[0, 2]) and np.all(tr[:, 4] == tr[0, 4])
        assert np.mean(np.diff(tr[:, 0]) != 0) > 0.2  # phi moves (Metropolis step)
        assert ref["accepted"].mean() > 0.5


def test_theta_update_with_level_move_matches_oracle():
    from paper_1603_08114_amd._lib import RSV_FLAG_LEVEL_MOVE
    Ts, C = [1500, 5000], 2
    thetas = synth.draw_batch_thetas(len(Ts), 3)
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, thetas=thetas, flags=RSV_FLAG_LEVEL_MOVE)
    st = smp.theta_update(sweep=4).cpu().numpy()
    th_gpu = smp.theta.cpu().numpy()
    h_gpu = smp.h.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        mv = oracle.level_move(h0[sl], th[c], ys[s] ** 2, smp.pb.seed, 4, c)
        assert mv["flags"] & 2
        ref_st = oracle.suffstats(mv["h"], rs[s], mv["theta"]["mu"], mv["theta"]["xi"])
        np.testing.assert_allclose(st[c], ref_st, rtol=1e-10, atol=1e-10 * np.abs(ref_st).max())
        ref_th, _ = oracle.theta_update(sl.stop - sl.start, ref_st, mv["theta"], smp.pb.seed, 4, c)
        got = dict(zip(oracle.THETA_KEYS, th_gpu[c]))
        for key in oracle.THETA_KEYS:
            assert got[key] == pytest.approx(ref_th[key], rel=1e-10, abs=1e-13), (c, key)
        assert rel_inf(h_gpu[sl], mv["h"]) <= 1e-13


def test_linear_gaussian_terms_f64():
    k, dt = 20, 0.05
    smp, offsets, ys, rs, h0, th = sampler([1000], 1, k=k, terms=RSV_TERM_RV)
    dh, acc = smp.trajectory(5, (k, dt))
    ref = oracle.trajectory(h0, ys[0] ** 2, rs[0], TH, k, dt, seed=smp.pb.seed, sweep=5,
                            terms=oracle.TERM_RV)
    assert abs(dh.item() - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
    assert rel_inf(smp.h.cpu().numpy(), ref["h"]) <= 1e-12


@pytest.mark.parametrize("Ts,C", [([1000], 1), ([513, 4000, 3], 2)])
def test_theta_update_and_statistics(Ts, C):
    thetas = synth.draw_batch_thetas(len(Ts), 77)
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, thetas=thetas)
    st = smp.theta_update(sweep=9).cpu().numpy()
    th_gpu = smp.theta.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        ref_st = oracle.suffstats(h0[sl], rs[s], th[c]["mu"], th[c]["xi"])
        np.testing.assert_allclose(st[c], ref_st, rtol=1e-12, atol=1e-12 * np.abs(ref_st).max())
        ref_th, _ = oracle.theta_update(sl.stop - sl.start, ref_st, th[c], smp.pb.seed, 9, c)
        got = dict(zip(oracle.THETA_KEYS, th_gpu[c]))
        for key in oracle.THETA_KEYS:
            assert got[key] == pytest.approx(ref_th[key], rel=1e-10, abs=1e-14), (c, key)


def _resync_builder(offsets, ys, rs, C, seed, k, **kw):
    """A fresh context (rsv_hmc_init) at a given state, for sweeps_with_resync."""
    def build(h, th):
        return api.RSVSampler(offsets, np.concatenate(ys), np.concatenate(rs), h, th,
                              chains_per_series=C, max_steps=k, seed=seed, **kw)
    return build


def oracle_ref(h0, th0, y2, r, k, dt, n, first, **kw):
    """The oracle chain (n sweeps from sweep `first`, h after every sweep),
    with what the parity helper needs to measure its sensitivity."""
    ref = oracle.run(h0, th0, y2, r, k, dt, n, first_sweep=first, keep_h=True, **kw)

    def step(h, th, i):
        o = oracle.run(h, th, y2, r, k, dt, 1, first_sweep=first + i, **kw)
        return o["h"], o["theta"], bool(o["accepted"][0]), float(o["dH"][0])
    ref.update(h0=np.asarray(h0, np.float64), theta0=dict(th0), step=step)
    return ref


def sweep_parity(Ts, C, k, dt, n, first, thetas=None, data_seed=105, state_jitter=0.05,
                 jitter=0.0, moves=0, terms=3, integrator=oracle.INT_LEAPFROG, flags=0):
    """Every chain of a multi-series problem against its oracle chain over n
    sweeps (theta updated), resynced at near-ties.  Returns the oracle runs."""
    offsets, ys, rs, hs = make_series(Ts, data_seed, thetas)
    h0 = state_from(hs, C, state_jitter)
    th = [thetas[s] if thetas else TH for s in range(len(Ts)) for _ in range(C)]
    slices = [sl for _, sl in chain_slices(offsets, C)]
    refs = [oracle_ref(h0[sl], th[c], ys[s] ** 2, rs[s], k, dt, n, first, seed=5, chain=c,
                       jitter=jitter, moves=moves, terms=terms, integrator=integrator)
            for c, (s, sl) in enumerate(chain_slices(offsets, C))]
    build = _resync_builder(offsets, ys, rs, C, 5, k, dtau_jitter=jitter, terms=terms,
                            flags=flags)
    n_ties, smp = sweeps_with_resync(build, h0, th, slices, refs, 5, first, n, (k, dt))
    if smp is not None:  # h after every sweep, the last included, was compared above
        smp.close()
    return refs


@pytest.mark.slow
def test_sweep_accept_sequence_single_series():
    """The single-series workload in full: T = 1000, k = 20, dtau = 0.05, 500
    burn-in + 5000 sweeps, theta every sweep.  Accept decisions, dH and theta
    of every sweep, and h after every sweep (rel <= 1e-10), equal the oracle's;
    a decision that differs inside the near-tie window is logged and the GPU
    chain is resynced to the oracle's state (rsv_hmc_init), so no sweep goes
    unchecked."""
    k, dt, n = 20, 0.05, 5500
    offsets, ys, rs, hs = make_series([1000], 105)
    h0 = hs[0]
    ref = oracle_ref(h0, TH, ys[0] ** 2, rs[0], k, dt, n, 0, seed=5)
    n_ties, smp = sweeps_with_resync(_resync_builder(offsets, ys, rs, 1, 5, k), h0, [TH],
                                     [slice(0, 1000)], [ref], 5, 0, n, (k, dt))
    print(f"near-ties resynced: {n_ties}; acceptance {ref['accepted'].mean():.3f}")
    assert ref["accepted"].mean() > 0.5
    if smp is not None:
        assert rel_inf(smp.h.cpu().numpy(), ref["h"]) <= 1e-10


def test_sweep_batched_chains_match_oracle():
    Ts, C, k, dt, n = [600, 1300, 2500], 2, 30, 0.04, 60
    thetas = synth.draw_batch_thetas(len(Ts), 5)
    offsets, ys, rs, hs = make_series(Ts, 105, thetas)
    h0 = state_from(hs, C, 0.02)
    th = [thetas[s] for s in range(len(Ts)) for _ in range(C)]
    slices = [sl for _, sl in chain_slices(offsets, C)]
    refs = [oracle_ref(h0[sl], th[c], ys[s] ** 2, rs[s], k, dt, n, 100, seed=5, chain=c)
            for c, (s, sl) in enumerate(chain_slices(offsets, C))]
    n_ties, smp = sweeps_with_resync(_resync_builder(offsets, ys, rs, C, 5, k), h0, th, slices,
                                     refs, 5, 100, n, (k, dt))
    if smp is not None:
        h_end = smp.h.cpu().numpy()
        for c, sl in enumerate(slices):
            assert rel_inf(h_end[sl], refs[c]["h"]) <= 1e-10


def test_sweep_is_deterministic():
    k, dt = 20, 0.05
    a, *_ = sampler([2000], 2, k=k)
    b, *_ = sampler([2000], 2, k=k)
    oa = a.sweep(0, 20, (k, dt))
    ob = b.sweep(0, 20, (k, dt))
    assert torch.equal(a.h, b.h)
    assert torch.equal(oa["theta"], ob["theta"])


@pytest.mark.parametrize("precision", [RSV_F64, RSV_F32_MIXED])
def test_two_stream_sweeps_equal_one_stream_sweeps(precision):
    """A context made by rsv_hmc_init runs the chains of rsv_hmc_sweep in two
    groups on two streams; a static context (rsv_hmc_init_static) runs them
    on its one stream.  Every output is the same bit for bit: h after every
    sweep, dH, decisions, theta, and the batch sums of h and h^2."""
    Ts, C, k, dt = [1000, 37, 2048, 1501, 700], 3, 20, 0.05
    offsets, ys, rs, hs = make_series(Ts, 41)
    h0 = state_from(hs, C, 0.05)
    th = [TH for _ in range(len(Ts) * C)]
    outs = []
    for static in (True, False):
        smp = api.RSVSampler(offsets, np.concatenate(ys), np.concatenate(rs), h0, th,
                             chains_per_series=C, precision=precision, max_steps=k, seed=9,
                             static_workspace=static)
        a = smp.sweep(0, 9, (k, dt), record=("delta_h", "accepted", "theta"), record_h=True)
        b = smp.sweep(9, 10, (k, dt), record=("accepted",), batch_len=4)
        outs.append((a, b, smp.h.clone(), smp.theta.clone()))
        smp.close()
    (a1, b1, h1, t1), (a2, b2, h2, t2) = outs
    for key in a1:
        assert torch.equal(a1[key], a2[key]), key
    for key in b1:
        assert torch.equal(b1[key], b2[key]), key
    assert torch.equal(h1, h2) and torch.equal(t1, t2)
    assert bool(a1["accepted"].any())


@pytest.mark.parametrize("terms", [3, 1])
def test_f32_mixed_trajectory_error_vs_f64(terms):
    """FP32 leapfrog, FP64 dH: error against the FP64 oracle on identical
    momenta, for the RSV model and the plain SV model (return term only).
    Bound derived from FP32 rounding (u = 6e-8) accumulated over k steps of a
    stable integrator on O(1) values."""
    k, dt = 20, 0.05
    smp, offsets, ys, rs, h0, th = sampler([1000, 2500], 1, k=k, precision=RSV_F32_MIXED,
                                           terms=terms)
    rng = np.random.default_rng(8)
    p0 = rng.standard_normal(smp.n_state)
    dh, acc = smp.trajectory(1, (k, dt), p0=p0, log_u=np.full(smp.n_chains, -50.0))
    h32 = smp.h.cpu().numpy().astype(np.float64)
    h0_32 = h0.astype(np.float32).astype(np.float64)
    for c, (s, sl) in enumerate(chain_slices(offsets, 1)):
        h1, p1 = oracle.leapfrog(h0_32[sl], p0[sl].astype(np.float32).astype(np.float64),
                                 ys[s] ** 2, rs[s], TH, k, dt, terms=terms)
        dH = oracle.delta_h(h0_32[sl], p0[sl].astype(np.float32).astype(np.float64), h1, p1,
                            ys[s] ** 2, rs[s], TH, terms=terms)
        assert np.max(np.abs(h32[sl] - h1)) <= 2e-5
        assert abs(dh[c].item() - dH) <= 2e-3 * np.sqrt(sl.stop - sl.start) / 30
    assert bool(acc.all())


def test_invalid_theta_rejected_at_init():
    offsets, ys, rs, hs = make_series([100], 1)
    with pytest.raises(api.RSVError) as e:
        api.RSVSampler(offsets, ys[0], rs[0], hs[0], dict(TH, phi=1.0), max_steps=10)
    assert e.value.status == -1


def test_nonfinite_state_rejected_at_init():
    offsets, ys, rs, hs = make_series([100], 1)
    h = hs[0].copy()
    h[17] = np.nan
    with pytest.raises(api.RSVError):
        api.RSVSampler(offsets, ys[0], rs[0], h, TH, max_steps=10)


def test_unstable_step_rejects_without_failure():
    smp, offsets, ys, rs, h0, th = sampler([800], 1, k=10)
    dh, acc = smp.trajectory(0, (10, 10.0))
    assert acc.item() == 0
    np.testing.assert_array_equal(smp.h.cpu().numpy(), h0)
    st, n_nonfinite = smp.check()
    assert st == 0 and n_nonfinite in (0, 1)


def test_poisoned_state_reported_by_check():
    smp, *_ = sampler([800], 1, k=10)
    smp.h[5] = float("nan")
    st, _ = smp.check()
    assert st == -5


@pytest.mark.parametrize("Ts,flags", [([800], 0), ([800], 1), ([5000, 700], 0)])
def test_poisoned_state_returned_by_the_next_call(Ts, flags):
    """A non-finite value written into the state is flagged by the kernels of
    the next sweep (resident or per-kernel path), that sweep's trajectory is
    rejected and theta is kept; the call after it returns RSV_ENONFINITE
    without running; once the state is repaired, rsv_hmc_check clears the
    flag and sweeps run again."""
    from paper_1603_08114_amd._lib import RSV_ENONFINITE
    k, dt = 10, 0.05
    smp, offsets, ys, rs, h0, th = sampler(Ts, 1, k=k, flags=flags)
    smp.sweep(0, 3, (k, dt), update_theta=True, record=())
    torch.cuda.synchronize()
    good_h, good_th = smp.h.clone(), smp.theta.clone()
    smp.h[17] = float("nan")
    out = smp.sweep(3, 2, (k, dt), update_theta=True, record=("accepted",))
    torch.cuda.synchronize()
    assert out["accepted"][:, 0].sum().item() == 0  # the poisoned chain rejects
    assert torch.equal(smp.theta[0], good_th[0])    # and keeps theta
    bad = smp.h.clone()
    with pytest.raises(api.RSVError) as e:
        smp.sweep(5, 1, (k, dt), update_theta=True, record=())
    assert e.value.status == RSV_ENONFINITE
    with pytest.raises(api.RSVError) as e:
        smp.trajectory(5, (k, dt))
    assert e.value.status == RSV_ENONFINITE
    assert torch.equal(smp.h.isnan(), bad.isnan())   # nothing ran
    smp.h[17] = good_h[17]
    st, _ = smp.check()
    assert st == 0
    smp.sweep(5, 2, (k, dt), update_theta=True, record=())
    torch.cuda.synchronize()
    assert smp.check()[0] == 0


@pytest.mark.parametrize("Ts,flags", [([700, 1500], 0), ([700, 1000], 0), ([700, 1000], 1)])
def test_batch_mean_accumulators_match_recorded_trace(Ts, flags):
    """Per-kernel sweeps (the next trajectory accumulates the previous state,
    the last state by a separate pass) and resident sweeps (all chains fit
    one tile; flags 0) against the recorded trace.  Both sum the states of a
    batch in FP32 and add the batch to the FP64 arrays."""
    k, dt, n, bl = 20, 0.05, 30, 7
    smp, offsets, ys, rs, h0, th = sampler(Ts, 2, k=k, flags=flags)
    out = smp.sweep(0, n, (k, dt), update_theta=True, record=(), record_h=True, batch_len=bl)
    h = out["h"].cpu().numpy()
    bs = out["h_batch_sum"].cpu().numpy()
    tol = 4e-7 * bl * np.abs(h).max()
    for b in range(bs.shape[0]):
        ref = np.zeros(h.shape[1])
        for i in range(b * bl, min(n, (b + 1) * bl)):
            ref += h[i]
        np.testing.assert_allclose(bs[b], ref, rtol=0, atol=tol)
    sq = np.zeros(h.shape[1])
    for i in range(n):
        sq += h[i] * h[i]
    np.testing.assert_allclose(out["h_sq_sum"].cpu().numpy(), sq, rtol=4e-7 * n)


RESIDENT_CASES = [
    # precision, jitter, flags, tile shape, series lengths, chains per series, k per series
    (RSV_F64, 0.0, 0, (8, 4), [1000, 37, 2048, 1501], 3, [20]),
    (RSV_F32_MIXED, 0.0, 0, (8, 4), [1000, 37, 2048, 1501], 3, [20]),
    (RSV_F64, 0.3, 2, (8, 4), [1000, 37, 2048, 1501], 3, [20]),
    (RSV_F32_MIXED, 0.3, 2, (8, 4), [1000, 37, 2048, 1501], 3, [20]),
    # multi-tile chains of single-wavefront tiles, long and short packed together
    (RSV_F32_MIXED, 0.0, 0, (8, 1), [8000, 513, 3, 4999, 1024, 7000, 64, 2500], 2, [20]),
    (RSV_F32_MIXED, 0.0, 0, (16, 1), [8000, 513, 3, 4999, 1024, 7000, 64, 2500], 2, [20]),
    (RSV_F64, 0.0, 0, (4, 1), [4096, 300, 2049, 17, 3100], 2, [20]),
    (RSV_F64, 0.0, 0, (4, 4), [9000, 300, 1000, 17, 1500], 3, [20]),
    # different step counts per series in one bin
    (RSV_F32_MIXED, 0.2, 2, (8, 1), [6000, 900, 3000, 40, 2222], 2, [20, 12, 20, 12, 12]),
]


@pytest.mark.parametrize("precision,dtau_jitter,flags,shape,Ts,C,ks", RESIDENT_CASES)
def test_resident_sweeps_equal_per_kernel_sweeps(precision, dtau_jitter, flags, shape, Ts, C,
                                                 ks):
    """With RSV_FLAG_RESIDENT, whole chains packed into bins run every sweep
    of a call in one launch; every record (dH, decisions, theta, h after
    every sweep, FP32-then-FP64 batch sums, final state) must equal the one-
    launch-per-kernel-per-sweep path of the same tile shape bit for bit."""
    from paper_1603_08114_amd._lib import RSV_FLAG_RESIDENT
    n, dt = 30, 0.04
    ks = ks * len(Ts) if len(ks) == 1 else ks
    lf = [(k, dt) for k in ks]
    thetas = synth.draw_batch_thetas(len(Ts), 9)
    offsets, ys, rs, hs = make_series(Ts, 300, thetas)
    h0 = state_from(hs, C, 0.02)
    th = [thetas[s] for s in range(len(Ts)) for _ in range(C)]
    outs = []
    for path in (0, RSV_FLAG_RESIDENT):
        smp = api.RSVSampler(offsets, np.concatenate(ys), np.concatenate(rs), h0, th,
                             chains_per_series=C, precision=precision, max_steps=max(ks), seed=4,
                             flags=flags | path, dtau_jitter=dtau_jitter, sites_per_lane=shape[0],
                             waves_per_tile=shape[1])
        o = smp.sweep(10, n, lf, update_theta=True, record_h=True, batch_len=7)
        o["state"] = smp.h.clone()
        o["theta_final"] = smp.theta.clone()
        outs.append(o)
    for key in ("delta_h", "accepted", "theta", "h", "state", "theta_final", "h_batch_sum",
                "h_sq_sum"):
        a, b = outs[0][key], outs[1][key]
        if a.is_floating_point():  # a diverged trajectory gives NaN on both paths
            assert torch.equal(a.isnan(), b.isnan()), key
            a, b = a.nan_to_num(nan=0.0), b.nan_to_num(nan=0.0)
        assert torch.equal(a, b), key
    assert outs[0]["accepted"].float().mean() > 0.3


def test_resident_sweeps_without_theta_update_and_with_mass():
    """Fixed theta (update_theta = 0) and a diagonal mass on the resident path."""
    from paper_1603_08114_amd._lib import RSV_FLAG_RESIDENT
    Ts, C, k, dt, n = [3000, 700, 41], 2, 15, 0.05, 20
    thetas = synth.draw_batch_thetas(len(Ts), 12)
    offsets, ys, rs, hs = make_series(Ts, 310, thetas)
    h0 = state_from(hs, C, 0.02)
    th = [thetas[s] for s in range(len(Ts)) for _ in range(C)]
    lm = (0.3 * np.random.default_rng(2).standard_normal(int(offsets[-1]))).astype(np.float32)
    for precision, shape in ((RSV_F32_MIXED, (8, 1)), (RSV_F64, (4, 4))):
        outs = []
        for path in (0, RSV_FLAG_RESIDENT):
            smp = api.RSVSampler(offsets, np.concatenate(ys), np.concatenate(rs), h0, th,
                                 chains_per_series=C, precision=precision, max_steps=k, seed=6,
                                 flags=path, log_mass=lm, sites_per_lane=shape[0],
                                 waves_per_tile=shape[1])
            o = smp.sweep(0, n, (k, dt), update_theta=False, record_h=True, batch_len=4)
            o["state"] = smp.h.clone()
            outs.append(o)
        for key in ("delta_h", "accepted", "theta", "h", "state", "h_batch_sum", "h_sq_sum"):
            assert torch.equal(outs[0][key], outs[1][key]), (precision, key)
        assert torch.equal(outs[0]["theta"][-1], outs[0]["theta"][0])


def test_autotuner_picks_a_compiled_shape_and_caches(tmp_path):
    from paper_1603_08114_amd import autotune
    offsets, ys, rs, hs = make_series([3000, 700], 21)
    th = [TH, TH]
    cache = str(tmp_path / "shapes.json")
    S, NW, table = autotune.best_shape(offsets, np.concatenate(ys), np.concatenate(rs),
                                       np.concatenate(hs), th, (30, 0.04), cache_path=cache,
                                       n_sweeps=3)
    assert (S, NW) in autotune.SHAPES[RSV_F64] and len(table) == len(autotune.SHAPES[RSV_F64])
    assert min(table.values()) == table[f"{S},{NW}"]
    S2, NW2, _ = autotune.best_shape(offsets, np.concatenate(ys), np.concatenate(rs),
                                     np.concatenate(hs), th, (30, 0.04), cache_path=cache)
    assert (S2, NW2) == (S, NW)


def test_tile_shapes_give_the_same_trajectory():
    """The per-site arithmetic does not depend on the tiling: h after a
    trajectory is bitwise equal across tile shapes."""
    k, dt = 30, 0.03
    outs = []
    for S, NW in [(4, 1), (8, 1), (4, 2), (4, 4), (4, 8), (8, 2), (8, 4), (8, 8)]:
        smp, offsets, ys, rs, h0, th = sampler([5000, 1200], 2, k=k, S=S, NW=NW)
        p0 = np.random.default_rng(2).standard_normal(h0.size)
        smp.trajectory(1, (k, dt), p0=p0, log_u=np.full(smp.n_chains, -50.0))
        outs.append(smp.h.cpu().numpy())
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_fp32_tile_shapes_agree():
    """FP32-mixed: h after a trajectory is bitwise equal across tile shapes
    (the FP32 loop's arithmetic does not depend on the tiling), and dH agrees
    to rounding (its tile partials are grouped by the tiling), over enough
    tiles (800 000 sites) that the wavefronts of a tile run at different
    paces: the tile's LDS stage is shared by them."""
    k, dt = 30, 0.03
    outs = []
    for S, NW in [(8, 1), (8, 2), (8, 4), (8, 8), (16, 1), (16, 2), (16, 4)]:
        smp, offsets, ys, rs, h0, th = sampler([200000, 200000], 2, k=k, S=S, NW=NW,
                                               precision=RSV_F32_MIXED)
        p0 = np.random.default_rng(3).standard_normal(h0.size)
        dh, acc = smp.trajectory(1, (k, dt), p0=p0, log_u=np.full(smp.n_chains, -1e9))
        outs.append((smp.h.cpu().numpy(), dh.cpu().numpy(), acc.cpu().numpy()))
        smp.close()
    for h, dh, acc in outs:  # every finite dH is accepted at ln u = -1e9
        assert np.all(np.isfinite(dh)) and bool(acc.all())
        np.testing.assert_array_equal(h, outs[0][0])
        np.testing.assert_allclose(dh, outs[0][1], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("S,NW,k,dt", [(4, 1, 123, 0.004), (8, 1, 251, 0.002), (8, 4, 1, 0.3),
                                       (4, 4, 2, 0.2)])
def test_extreme_step_counts(S, NW, k, dt):
    """The largest k a tile shape accepts (halo = all but 8 sites of the tile)
    and single/double steps, over ragged chains spanning several tiles."""
    Ts, C = [1000, 300, 3], 2
    smp, offsets, ys, rs, h0, th = sampler(Ts, C, k=k, S=S, NW=NW)
    dh, acc = smp.trajectory(9, (k, dt))
    h_gpu, dh, acc = smp.h.cpu().numpy(), dh.cpu().numpy(), acc.cpu().numpy()
    for c, (s, sl) in enumerate(chain_slices(offsets, C)):
        ref = oracle.trajectory(h0[sl], ys[s] ** 2, rs[s], th[c], k, dt, seed=smp.pb.seed,
                                sweep=9, chain=c)
        assert abs(dh[c] - ref["dH"]) <= 1e-9 * max(1.0, abs(ref["dH"]))
        if abs(ref["dH"] + oracle.log_u(smp.pb.seed, 9, c)) > NEAR_TIE:
            assert bool(acc[c]) == ref["accepted"]
            assert rel_inf(h_gpu[sl], ref["h"]) <= 1e-12


def test_many_minimum_length_chains():
    """4096 chains of T = 3 (one partial lane each), several sweeps with theta."""
    sweep_parity([3] * 1024, 4, 10, 0.1, 12, 0)
