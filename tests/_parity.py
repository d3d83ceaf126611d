"""Sweep-by-sweep parity of GPU chains with oracle chains, with resync at
near-ties (test-only helper).

Both sides draw the same counter-based random numbers, so a GPU chain and the
oracle chain from the same state take the same accept/reject decisions and
the same theta draws.  The one legitimate difference is a Metropolis test
whose margin |dH + ln u| is below the rounding difference of the two dH sums
(the near-tie window 1e-9): there the chains may take different decisions.
Each such sweep is logged, and the GPU context is re-created through
rsv_hmc_init at the oracle's state after that sweep (other chains at their
GPU state), so every later sweep is still compared.
"""
import numpy as np

import oracle

NEAR_TIE = 1e-9
DIVERGED = 1e3  # a dH this large rejects for every uniform (ln u > -37)
THETA_KEYS = oracle.THETA_KEYS
# theta bar: |d theta_i| <= 1e-10 max(|theta_i|, floor_i); floor 1 for the
# locations mu and xi, none for phi and the variances
THETA_REL_FLOOR = np.array([0.0, 1.0, 1.0, 0.0, 0.0])


def _rel_inf(a, b):
    return np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b)))


def oracle_sensitivity(ref, step, trials=4, eps=1e-14, seed=0):
    """How strongly an oracle chain amplifies rounding-level differences:
    the chain is re-run with its state perturbed by eps (relative, random
    sign) after every sweep, and the largest change of dH (absolute), of
    theta (relative, with the floors of the theta bar) and of h (relative
    inf-norm) is returned per sweep, over trials whose decisions stay those
    of `ref`.  step(h, theta, i) -> (h, theta dict, accepted, dH) runs sweep
    i of the oracle chain."""
    n = len(ref["accepted"])
    d_dh, d_th, d_h = np.zeros(n), np.zeros(n), np.zeros(n)
    rng = np.random.default_rng(seed)
    for _ in range(trials):
        h, th = ref["h0"] * (1 + eps * rng.choice([-1.0, 1.0], ref["h0"].size)), ref["theta0"]
        for i in range(n):
            h, th, acc, dh = step(h, th, i)
            if acc != bool(ref["accepted"][i]):
                break
            if np.isfinite(dh) and np.isfinite(ref["dH"][i]):
                d_dh[i] = max(d_dh[i], abs(dh - ref["dH"][i]))
            t = np.array([th[k] for k in THETA_KEYS])
            want = ref["theta_trace"][i]
            d_th[i] = max(d_th[i], np.max(np.abs(t - want) / np.maximum(np.abs(want),
                                                                         THETA_REL_FLOOR)))
            d_h[i] = max(d_h[i], _rel_inf(h, ref["h_trace"][i]))
            h = h * (1 + eps * rng.choice([-1.0, 1.0], h.size))
    return d_dh, d_th, d_h


def first_divergence(gpu_acc, gpu_dh, gpu_theta, gpu_h, ref, seed, chain, first, start,
                     h_tol=1e-10, log=print):
    """Compare sweeps [start, start + len(gpu_acc)) of one chain with the
    oracle run `ref` (made with keep_h=True from the chain's state before
    sweep `first`).  Returns the index (into ref) of the first near-tie at
    which the decisions differ, or None; asserts equality everywhere before.

    Bars: dH 1e-9 (relative above 1), theta 1e-10 relative (mu, xi: of
    max(|value|, 1)), h 1e-10 relative, decisions equal outside the near-tie
    window 1e-9.  Where a chain amplifies rounding differences faster than
    that (short, ill-conditioned chains), each bar of a sweep becomes 10
    times what the oracle chain itself shows under 1e-14 perturbations of its
    state after every sweep (oracle_sensitivity, computed only for such
    chains; needs ref["step"], ref["h0"] and ref["theta0"]); each such sweep
    is logged."""
    sens = None

    def sensitivity(i):
        nonlocal sens
        assert "step" in ref, (chain, first + i)
        if sens is None:
            sens = oracle_sensitivity(ref, ref["step"])
        return sens[0][i], sens[1][i], sens[2][i]

    for j in range(len(gpu_acc)):
        i = start + j
        lu = oracle.log_u(seed, first + i, chain)
        if bool(gpu_acc[j]) != bool(ref["accepted"][i]):
            margin = abs(ref["dH"][i] + lu)
            if margin >= NEAR_TIE:
                s_dh = sensitivity(i)[0]
                log(f"chain {chain} sweep {first + i}: decision differs at margin {margin:.1e}; "
                    f"the oracle chain amplifies 1e-14 to dH {s_dh:.1e}")
                assert margin < 10 * s_dh, (
                    f"chain {chain} sweep {first + i}: decision differs outside the near-tie "
                    f"window (dH oracle {ref['dH'][i]!r}, GPU {gpu_dh[j]!r}, ln u {lu!r})")
            return i
        regular = [np.isfinite(v) and abs(v) < DIVERGED for v in (gpu_dh[j], ref["dH"][i])]
        if all(regular):
            e_dh = abs(gpu_dh[j] - ref["dH"][i]) / max(1.0, abs(ref["dH"][i]))
        else:
            # a diverged trajectory: the two exponentials saturate or overflow
            # differently far outside the sampled range, so the dH values are
            # not comparable; both must reject with dH non-finite or beyond
            # any ln u (> -37)
            for v in (gpu_dh[j], ref["dH"][i]):
                assert not (np.isfinite(v) and v < DIVERGED), (chain, first + i, gpu_dh[j],
                                                               ref["dH"][i])
            assert not gpu_acc[j] and not ref["accepted"][i], (chain, first + i)
            e_dh = 0.0
        want = ref["theta_trace"][i]
        e_th = np.max(np.abs(gpu_theta[j] - want) / np.maximum(np.abs(want), THETA_REL_FLOOR))
        e_h = _rel_inf(gpu_h[j], ref["h_trace"][i]) if gpu_h is not None else 0.0
        if e_dh > 1e-9 or e_th > 1e-10 or e_h > h_tol:
            s_dh, s_th, s_h = sensitivity(i)
            log(f"chain {chain} sweep {first + i}: dH {e_dh:.1e}, theta {e_th:.1e}, h {e_h:.1e} "
                f"beyond the bars; the oracle chain amplifies 1e-14 to dH {s_dh:.1e}, "
                f"theta {s_th:.1e}, h {s_h:.1e}")
            assert (e_dh <= max(1e-9, 10 * s_dh) and e_th <= max(1e-10, 10 * s_th)
                    and e_h <= max(h_tol, 10 * s_h)), (chain, first + i, e_dh, e_th, e_h)
    return None


def sweeps_with_resync(build, h0, thetas, slices, refs, seed, first, n, lf, log=print):
    """Run n sweeps on the GPU and compare every chain with its oracle run.

    build(h_state, theta_list) -> a fresh RSVSampler (rsv_hmc_init) at that
    state; slices[c] is chain c's slice of the state vector; refs[c] the
    oracle run of chain c (keep_h=True).  Returns (number of resyncs, the
    last sampler) after asserting parity over all n sweeps."""
    h = np.array(h0, dtype=np.float64, copy=True)
    th = [dict(t) for t in thetas]
    i0, ties = 0, []
    while True:
        smp = build(h, th)
        out = smp.sweep(first + i0, n - i0, lf, update_theta=True, record_h=True)
        acc = out["accepted"].cpu().numpy()
        dh = out["delta_h"].cpu().numpy()
        tht = out["theta"].cpu().numpy()
        hh = out["h"].cpu().numpy().astype(np.float64)
        div = {}
        for c, sl in enumerate(slices):
            d = first_divergence(acc[:, c], dh[:, c], tht[:, c], hh[:, sl], refs[c], seed, c,
                                 first, i0)
            if d is not None:
                div[c] = d
        if not div:
            return len(ties), smp
        i = min(div.values())
        # every chain matched up to sweep i; the ones that differ at i take the
        # oracle's state after it, the others keep the GPU state (identical up
        # to rounding)
        for c, sl in enumerate(slices):
            j = i - i0
            if div.get(c) == i:
                log(f"near-tie: chain {c} sweep {first + i}: dH={refs[c]['dH'][i]!r} "
                    f"ln u={oracle.log_u(seed, first + i, c)!r}; resync at the oracle state")
                ties.append((c, i))
                h[sl] = refs[c]["h_trace"][i]
                th[c] = dict(zip(THETA_KEYS, refs[c]["theta_trace"][i]))
            else:
                h[sl] = hh[j, sl]
                th[c] = dict(zip(THETA_KEYS, tht[j, c]))
        smp.close()
        i0 = i + 1
        if i0 >= n:
            return len(ties), None
