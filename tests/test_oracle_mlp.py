"""Pins of the learned-mass network oracle (oracle/mlp_oracle.py).

bfloat16 rounding against torch's CPU conversion; the forward pass against a
torch.nn.Sequential model of the same layers (FP64, and with torch's bfloat16
conversion at the rounding points) and against the closed form of a single
active path; gradients against torch autograd of that model and against
central finite differences of the FP64 (unrounded) loss; Adam against
torch.optim.Adam; GELU against its definition; feature windows against
direct indexing.
"""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def test_bf16_round_matches_torch_rne():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(M.bf16_round(x), ref)


def test_gelu_and_derivative():
    x = np.linspace(-6, 6, 1001)
    from scipy.stats import norm
    np.testing.assert_allclose(M.gelu(x), x * norm.cdf(x), rtol=1e-12, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(x), (M.gelu(x + h) - M.gelu(x - h)) / (2 * h),
                               rtol=1e-6, atol=1e-9)


def test_feature_window_clamps_to_the_series():
    T = 9
    y2 = np.arange(1, T + 1, dtype=float)
    lr = -np.arange(T, dtype=float)
    th = dict(phi=0.9, mu=-0.1, xi=0.2, sig2_eta=0.05, sig2_u=0.1)
    F = M.raw_features(y2, lr, th)
    assert F.shape == (T, M.N_IN)
    for t in range(T):
        for d in range(-5, 6):
            j = min(max(t + d, 0), T - 1)
            assert F[t, d + 5] == np.log(y2[j] + M.Y2_FLOOR)
            assert F[t, 11 + d + 5] == lr[j]
        assert list(F[t, 22:]) == [th[k] for k in M.THETA_KEYS]


def _problem(n=40, seed=1):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, M.N_IN_PAD))
    X[:, :M.N_IN] = rng.standard_normal((n, M.N_IN))
    return M.init_params(seed), X, rng.standard_normal(n)


def test_gradient_matches_finite_differences_fp64():
    p, X, y = _problem()
    g = M.grad(p, X, y, bf16=False)
    v = M.flatten(p)
    gv = M.flatten(g)
    rng = np.random.default_rng(5)
    idx = rng.choice(np.nonzero(np.abs(gv) > 1e-8)[0], 150, replace=False)
    for i in idx:
        h = 1e-6 * max(1.0, abs(v[i]))
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fd = (M.loss(M.unflatten(vp), X, y, False) - M.loss(M.unflatten(vm), X, y, False)) / (2 * h)
        assert abs(fd - gv[i]) <= 1e-6 * max(abs(gv[i]), 1e-3), (i, fd, gv[i])


def test_bf16_gradient_close_to_fp64_gradient():
    p, X, y = _problem(256)
    g64 = M.flatten(M.grad(p, X, y, bf16=False))
    g16 = M.flatten(M.grad(p, X, y, bf16=True))
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


def test_adam_matches_torch():
    p, X, y = _problem(64)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    s = {k: np.zeros_like(v) for k, v in p.items()}
    for step in range(1, 6):
        g = M.grad(p, X, y, bf16=False)
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
        M.adam(p, g, m, s, step, 1e-3)
        for k in p:
            np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    n = 2000
    X = np.zeros((n, M.N_IN_PAD))
    X[:, :M.N_IN] = rng.standard_normal((n, M.N_IN))
    target = np.tanh(X[:, 0] - 0.5 * X[:, 12]) + 0.3 * X[:, 24]
    p = M.init_params(0)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    s = {k: np.zeros_like(v) for k, v in p.items()}
    l0 = M.loss(p, X, target)
    for step in range(1, 301):
        M.adam(p, M.grad(p, X, target), m, s, step, 3e-3)
    assert M.loss(p, X, target) < 0.1 * l0


# --- forward and gradient against an independent torch.nn model ---------------
def _torch_net(p):
    """The network as torch.nn layers (FP64): Linear(32, 64), GELU (erf form),
    Linear(64, 64), GELU, Linear(64, 1), with the oracle's parameters."""
    nn = torch.nn
    net = nn.Sequential(nn.Linear(M.N_IN_PAD, M.HIDDEN), nn.GELU(approximate="none"),
                        nn.Linear(M.HIDDEN, M.HIDDEN), nn.GELU(approximate="none"),
                        nn.Linear(M.HIDDEN, 1)).double()
    with torch.no_grad():
        net[0].weight.copy_(torch.tensor(p["W1"].T))
        net[0].bias.copy_(torch.tensor(p["b1"]))
        net[2].weight.copy_(torch.tensor(p["W2"].T))
        net[2].bias.copy_(torch.tensor(p["b2"]))
        net[4].weight.copy_(torch.tensor(p["w3"][None, :]))
        net[4].bias.copy_(torch.tensor(p["b3"]))
    return net


def _torch_bf16(t):
    """torch's own FP64 -> FP32 -> bfloat16 conversion (round to nearest even)."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def _params_with_biases(seed):
    p = M.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = 0.1 * rng.standard_normal(M.HIDDEN)
    p["b2"] = 0.1 * rng.standard_normal(M.HIDDEN)
    p["b3"] = np.array([0.25])
    return p


def test_forward_fp64_matches_torch_nn():
    p = _params_with_biases(4)
    _, X, _ = _problem(300, seed=4)
    out, _ = M.forward(p, X, bf16=False)
    ref = _torch_net(p)(torch.tensor(X)).detach().numpy()[:, 0]
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-13)


def test_forward_bf16_matches_torch_with_bf16_rounding_points():
    """The rounding points: inputs, weights and both hidden activations in
    bfloat16, products and biases in wide precision."""
    p = _params_with_biases(6)
    _, X, _ = _problem(500, seed=6)
    net = _torch_net(p)
    F = torch.nn.functional
    with torch.no_grad():
        x = _torch_bf16(torch.tensor(X))
        h1 = _torch_bf16(net[1](F.linear(x, _torch_bf16(net[0].weight), net[0].bias)))
        h2 = _torch_bf16(net[3](F.linear(h1, _torch_bf16(net[2].weight), net[2].bias)))
        ref = F.linear(h2, _torch_bf16(net[4].weight), net[4].bias).numpy()[:, 0]
    out, _ = M.forward(p, X, bf16=True)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-12)
    # and the rounding matters: the unrounded network differs at the bf16 level
    out64, _ = M.forward(p, X, bf16=False)
    assert 1e-4 < np.max(np.abs(out - out64)) < 0.5


def test_forward_single_path_closed_form():
    """One input, one unit per layer: out = b3 + u gelu(v gelu(w x + b1) + b2)."""
    p = {k: np.zeros_like(v) for k, v in M.init_params(0).items()}
    w, v, u, b1, b2, b3 = 0.7, -1.3, 2.0, 0.2, 0.1, -0.4
    p["W1"][3, 5], p["W2"][5, 9], p["w3"][9] = w, v, u
    p["b1"][5], p["b2"][9], p["b3"][0] = b1, b2, b3
    x = np.linspace(-3, 3, 13)
    X = np.zeros((x.size, M.N_IN_PAD))
    X[:, 3] = x
    from scipy.stats import norm
    g = lambda z: z * norm.cdf(z)
    # the other units see only their (zero) biases: gelu(0) = 0
    expect = b3 + u * g(v * g(w * x + b1) + b2)
    out, _ = M.forward(p, X, bf16=False)
    np.testing.assert_allclose(out, expect, rtol=1e-13, atol=1e-14)


def test_gradient_fp64_matches_torch_autograd():
    p = _params_with_biases(8)
    _, X, y = _problem(200, seed=8)
    net = _torch_net(p)
    loss = torch.mean((net(torch.tensor(X))[:, 0] - torch.tensor(y)) ** 2)
    loss.backward()
    ref = dict(W1=net[0].weight.grad.numpy().T, b1=net[0].bias.grad.numpy(),
               W2=net[2].weight.grad.numpy().T, b2=net[2].bias.grad.numpy(),
               w3=net[4].weight.grad.numpy()[0], b3=net[4].bias.grad.numpy())
    g = M.grad(p, X, y, bf16=False)
    for k in ref:
        np.testing.assert_allclose(g[k], ref[k], rtol=1e-10, atol=1e-13, err_msg=k)
    assert M.loss(p, X, y, bf16=False) == pytest.approx(loss.item(), rel=1e-13)


def test_log_mass_clips_finite_outputs_only():
    """The oracle's log mass: finite outputs clipped to [-5, 5], non-finite
    ones passed on (the sampler's identity fallback handles them)."""
    p = M.init_params(4)
    X = np.zeros((50, 32))
    X[:, :27] = np.random.default_rng(2).standard_normal((50, 27))
    p["b3"][:] = 40.0
    assert np.all(M.log_mass(p, X, bf16=False) == 5.0)
    p["b3"][:] = np.inf
    out = M.log_mass(p, X, bf16=False)
    assert np.all(np.isinf(out))
