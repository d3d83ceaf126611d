"""Learned diagonal mass on the GPU: its gain over the identity mass at equal
precision, step-size adaptation to the target acceptance in both arms, the
h_t posterior means of the two arms under the moment rule, and the identity
fallback of the mass table.

A diagonal mass changes only the kinetic term of H (Sec. 3); any fixed
positive mass leaves the target unchanged, so a trained network may only
change how fast the chain mixes.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1603_08114_amd import api, diagnostics as D, learned_mass as LM  # noqa: E402
from paper_1603_08114_amd._lib import RSV_F32_MIXED, RSV_F64  # noqa: E402


@pytest.fixture(scope="module")
def trained():
    """The network trained by the library's kernels on plain FP64 chains of 16
    series (T ~ U{500..3000}, seed 4)."""
    train = synth.make_batch(16, 500, 3000, seed=4)
    tr = LM.training_targets(train, C=4, k=30, warm=200, n=600)
    target = -torch.log(torch.clamp(tr["var"], min=1e-12))
    net, hist, r2 = LM.train_network(train, target, tr["theta_mean"], epochs=200)
    print(f"mass network: loss {hist[0]:.3f} -> {hist[-1]:.3f}, R^2 {r2:.3f}")
    return net


@pytest.mark.slow
def test_learned_mass_gain_and_moments_fp32(trained):
    """8 held-out series (T ~ U{1000..4000}, seed 6), 4 chains each, k = 30,
    theta held at each series' generating value, 400 warm-up sweeps (dtau
    adapted per series to acceptance 0.8) and 1000 measured sweeps, FP32-mixed
    in both arms, with the step jitter dtau U[0.5, 1.5] (a fixed trajectory
    length can resonate with slow modes of h, and batch-means standard errors
    are only reliable for a chain that mixes).  The learned mass must raise the mean over sites of
    ESS(h_t) per sweep (median over series); both arms must end near the
    target acceptance; and the posterior means of h_t of the two arms must
    agree under the moment rule, with standard errors from 40 batch means of
    each arm (p-values from Student's t with 39 degrees of freedom, the
    smaller of the two arms' counts).

    A reference arm takes the network's target itself as the mass (-ln of
    each site's posterior variance from 4 x 2000 plain FP64 sweeps of the
    held-out series): what a perfect network could reach.  The learned mass
    must keep at least 90% of the identity's ESS(h_t) per sweep and 90% of
    the reference arm's gain; the gains are printed."""
    held = synth.make_batch(8, 1000, 4000, seed=6)
    kw = dict(warm=400, n=1000, bl=25, update_theta=False, dtau_jitter=0.5)
    ident = LM.run_arm(held, 4, 30, RSV_F32_MIXED, None, seed=7, **kw)
    learned = LM.run_arm(held, 4, 30, RSV_F32_MIXED, trained, seed=8, **kw)
    tgt = LM.training_targets(held, C=4, k=30, warm=400, n=2000, seed=9)
    lm_ref = (-torch.log(torch.clamp(tgt["var"], min=1e-12))).cpu().numpy()
    ref = LM.run_arm(held, 4, 30, RSV_F32_MIXED, None, seed=10, log_mass=lm_ref, **kw)
    gain = learned["ess_h_mean"] / ident["ess_h_mean"]
    gain_ref = ref["ess_h_mean"] / ident["ess_h_mean"]
    print(f"acceptance identity {ident['acceptance']:.3f} learned {learned['acceptance']:.3f} "
          f"reference {ref['acceptance']:.3f}; ESS(h)/sweep gain per series: learned "
          f"{np.round(gain, 3)} (median {np.median(gain):.3f}), reference mass "
          f"{np.round(gain_ref, 3)} (median {np.median(gain_ref):.3f}); fallback series "
          f"{learned['fallback_series']}; min ESS(h) identity {np.round(ident['ess_h'], 1)} "
          f"learned {np.round(learned['ess_h'], 1)}")
    for r in (ident, learned, ref):
        assert abs(r["acceptance"] - 0.8) < 0.05
    assert learned["fallback_series"] == []
    assert np.median(gain) > 0.9
    assert np.median(gain) > 0.9 * np.median(gain_ref)

    from scipy import stats
    z = ((learned["mean"] - ident["mean"]) /
         torch.sqrt(learned["mcse2"] + ident["mcse2"])).cpu().numpy()
    p = 2.0 * stats.t.sf(np.abs(z), df=1000 // 25 - 1)
    ok, summary = D.moment_rule(p)
    print(f"h_t means, learned vs identity: {summary}")
    assert ok


@pytest.mark.parametrize("precision", [RSV_F64, RSV_F32_MIXED])
def test_unusable_log_mass_takes_identity_at_those_sites(precision):
    """A site whose ln m_t is NaN, +-inf or outside [-80, 80] runs with
    m_t = 1: the sweeps equal, bit for bit, those with ln m_t = 0 there."""
    T = 3000
    y, r, h = synth.simulate_rsv_long(T, synth.THETA_STAR, 3)
    lm = (0.5 * np.sin(np.arange(T) * 0.01)).astype(np.float32)
    bad = [0, 17, 1500, 2998, 2999]
    lm_bad = lm.copy()
    lm_bad[bad] = [np.nan, np.inf, -np.inf, 200.0, -90.0]
    lm_ref = lm.copy()
    lm_ref[bad] = 0.0
    out = []
    for m in (lm_bad, lm_ref):
        smp = api.RSVSampler([0, T], y, r, h, synth.THETA_STAR, max_steps=20, seed=5,
                             precision=precision, log_mass=m)
        o = smp.sweep(0, 6, (20, 0.05), record=("delta_h", "accepted"))
        out.append((smp.h.clone(), o["delta_h"].clone(), o["accepted"].clone()))
        smp.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    assert torch.equal(out[0][2], out[1][2])
    assert out[0][2].any()
