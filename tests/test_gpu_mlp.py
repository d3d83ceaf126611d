"""Parity of the BF16-MFMA mass network kernels with the FP64 oracle that
emulates their rounding points (oracle/mlp_oracle.py).  Bars: forward
elementwise rel <= 1e-2, norm rel <= 1e-3; gradient norm rel <= 1e-3 and
elementwise rel <= 1e-2 above a floor of 1e-3 of each block's largest entry;
Adam rel <= 1e-5 (FP32 vs FP64); features equal except rare last-bit
differences of the bfloat16 rounding (FP64 log on both sides)."""
import numpy as np
import pytest

import synth
from oracle import mlp_oracle as M

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1603_08114_amd import mass  # noqa: E402


def bf16_bits_to_float(x16):
    u = x16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def series_data(Ts, seed):
    data = [synth.simulate_rsv(T, synth.THETA_STAR, seed + i) for i, T in enumerate(Ts)]
    thetas = synth.draw_batch_thetas(len(Ts), seed)
    off = np.concatenate([[0], np.cumsum(Ts)]).astype(np.int64)
    y = np.concatenate([d[0] for d in data])
    lr = np.concatenate([d[1] for d in data])
    return off, y, lr, thetas


def stats_of(off, y, lr, thetas):
    raw = np.concatenate([M.raw_features(y[off[s]:off[s + 1]] ** 2, lr[off[s]:off[s + 1]],
                                         thetas[s]) for s in range(len(thetas))])
    return raw, raw.mean(0), raw.std(0) + 1e-3


def test_features_match_oracle():
    off, y, lr, thetas = series_data([300, 11, 1000], 4)
    raw, mean, std = stats_of(off, y, lr, thetas)
    net = mass.MassNet(M.flatten(M.init_params(0)), mean, std)
    x = net.features(off, y, lr, synth.theta_array(thetas))
    got = bf16_bits_to_float(x)
    ref = np.zeros_like(got)
    ref[:, :M.N_IN] = M.bf16_round(M.standardise(raw, mean, std))
    exact = np.mean(got == ref)
    assert exact > 0.999, exact
    ulp = np.abs(ref) * 2.0 ** -7 + 1e-30
    assert np.all(np.abs(got - ref) <= ulp)
    assert np.all(got[:, M.N_IN:] == 0)


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, M.N_IN_PAD))
    X[:, :M.N_IN] = rng.standard_normal((n, M.N_IN))
    Xb = M.bf16_round(X)
    bits = (Xb.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)
    return Xb, torch.as_tensor(bits, device="cuda").contiguous()


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 4097])
def test_forward_matches_oracle(n):
    p = M.init_params(1)
    p["b1"][:] = 0.1
    p["b2"][:] = -0.05
    p["b3"][:] = 0.3
    Xb, xg = _inputs(n, n)
    net = mass.MassNet(M.flatten(p), np.zeros(27), np.ones(27))
    out = net.forward(xg).cpu().numpy().astype(np.float64)
    ref, _ = M.forward(p, Xb, bf16=True)
    assert np.max(np.abs(out - ref) / np.maximum(np.abs(ref), 1e-1)) <= 1e-2
    assert np.linalg.norm(out - ref) <= 1e-3 * np.linalg.norm(ref) + 1e-6
    clipped = net.forward(xg, clip=True).cpu().numpy()
    assert np.all(np.abs(clipped) <= 5.0)


@pytest.mark.parametrize("n,use_rows", [(64, False), (1000, False), (3001, True)])
def test_gradient_matches_oracle(n, use_rows):
    p = M.init_params(2)
    Xb, xg = _inputs(n, 7)
    target = np.random.default_rng(1).standard_normal(n)
    net = mass.MassNet(M.flatten(p), np.zeros(27), np.ones(27))
    tg = torch.as_tensor(target.astype(np.float32), device="cuda")
    rows = None
    sel = np.arange(n)
    if use_rows:
        sel = np.random.default_rng(3).permutation(n)[: n // 2]
        rows = torch.as_tensor(sel.astype(np.int32), device="cuda")
    g, loss = net.gradient(xg, tg, rows)
    ref = M.flatten(M.grad(p, Xb[sel], target.astype(np.float32).astype(np.float64)[sel], bf16=True))
    got = g.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"gradient: norm rel err {err:.2e}")
    assert err <= 1e-3, err
    # elementwise within each parameter block, above a floor of 1e-3 of the
    # block's largest entry (smaller entries are sums that cancel to below the
    # FP32 accumulation error of their terms)
    i = 0
    for name, shape in M.PARAM_SHAPES:
        n_el = int(np.prod(shape))
        r, gv = ref[i:i + n_el], got[i:i + n_el]
        i += n_el
        floor = 1e-3 * np.max(np.abs(r)) if np.any(r) else 1e-30
        big = np.abs(r) >= floor
        rel = np.abs(gv[big] - r[big]) / np.abs(r[big])
        print(f"  {name}: {big.sum()}/{n_el} entries above floor, max rel err {rel.max():.2e}")
        assert rel.max() <= 1e-2, (name, rel.max())
        assert np.all(np.abs(gv[~big] - r[~big]) <= 1e-2 * floor + 1e-5 * np.max(np.abs(r))), name
    ref_loss = M.loss(p, Xb[sel], target.astype(np.float32).astype(np.float64)[sel], bf16=True)
    assert loss.item() == pytest.approx(ref_loss, rel=1e-4)
    # padding rows of W1 get no gradient
    assert np.all(got[M.N_IN * M.HIDDEN:M.N_IN_PAD * M.HIDDEN] == 0)


def test_adam_matches_oracle():
    p = M.init_params(3)
    rng = np.random.default_rng(5)
    net = mass.MassNet(M.flatten(p), np.zeros(27), np.ones(27))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    s = {k: np.zeros_like(v) for k, v in p.items()}
    pf = M.unflatten(M.flatten(p).astype(np.float32).astype(np.float64))
    for step in range(1, 4):
        g = M.unflatten(rng.standard_normal(M.N_PARAMS).astype(np.float32).astype(np.float64))
        mass.rsv_mlp_adam(net.params, net.m, net.v,
                          torch.as_tensor(M.flatten(g).astype(np.float32), device="cuda"), step, 1e-3)
        M.adam(pf, g, m, s, step, 1e-3)
    np.testing.assert_allclose(net.params.cpu().numpy(), M.flatten(pf), rtol=1e-5, atol=1e-7)


def test_training_on_gpu_reduces_loss():
    n = 20000
    Xb, xg = _inputs(n, 11)
    target = np.tanh(Xb[:, 0] - 0.5 * Xb[:, 12]) + 0.3 * Xb[:, 24]
    net = mass.MassNet(M.flatten(M.init_params(0)), np.zeros(27), np.ones(27))
    tg = torch.as_tensor(target.astype(np.float32), device="cuda")
    hist = net.fit(xg, tg, epochs=8, batch=2048, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0], hist


def test_clip_passes_non_finite_outputs():
    """With the clip on, a finite output is clipped to [-5, 5] and a non-finite
    one (here every output, from a NaN output bias) is passed on unchanged,
    so that the identity fallback sees it; the oracle does the same."""
    p = M.init_params(1)
    p["b3"][:] = np.nan
    Xb, xg = _inputs(100, 3)
    net = mass.MassNet(M.flatten(p), np.zeros(27), np.ones(27))
    assert np.all(np.isnan(net.forward(xg, clip=True).cpu().numpy()))
    assert np.all(np.isnan(M.log_mass(p, Xb)))
