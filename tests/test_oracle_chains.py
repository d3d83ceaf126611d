"""oracle.chains: per-chain moments of segmented oracle runs equal those of
one unsegmented run (the segments continue the sweep counter and the state),
and the layout of the returned arrays."""
import numpy as np

import oracle
import synth
from oracle.chains import chain_moments


def test_segmented_chains_equal_one_run():
    Ts = [40, 65]
    off = np.concatenate([[0], np.cumsum(Ts)])
    data = [synth.simulate_rsv(T, synth.THETA_STAR, 20 + i) for i, T in enumerate(Ts)]
    y = np.concatenate([d[0] for d in data])
    lr = np.concatenate([d[1] for d in data])
    h0s = [d[2] for d in data]
    th = [synth.THETA_STAR, synth.THETA_STAR]
    C, k, dts, n_burn, n = 3, 10, [0.1, 0.08], 7, 23
    got = chain_moments(off, y, lr, h0s, th, C, k, dts, n_burn, n, seed=9, seg=5, threads=2)
    assert got["h_mean"].shape == (C, sum(Ts)) and got["theta_mean"].shape == (C, 10)
    for c in range(C):
        for s in range(2):
            y2 = y[off[s]:off[s + 1]] ** 2
            o = oracle.run(h0s[s], th[s], y2, lr[off[s]:off[s + 1]], k, dts[s], n_burn + n,
                           seed=9, chain=c, keep_h=True)
            ht = o["h_trace"][n_burn:]
            tt = o["theta_trace"][n_burn:]
            np.testing.assert_allclose(got["h_mean"][c, off[s]:off[s + 1]], ht.mean(0),
                                       rtol=1e-12, atol=1e-12)
            np.testing.assert_allclose(got["h_var"][c, off[s]:off[s + 1]], ht.var(0),
                                       rtol=1e-9, atol=1e-12)
            np.testing.assert_allclose(got["theta_mean"][c, 5 * s:5 * s + 5], tt.mean(0),
                                       rtol=1e-12)
            np.testing.assert_allclose(got["theta_var"][c, 5 * s:5 * s + 5], tt.var(0),
                                       rtol=1e-9, atol=1e-15)
