"""Pins of the learned-mass network oracle (oracle/mlp_oracle.py).

bfloat16 rounding against torch's CPU conversion; gradients against central
finite differences of the FP64 (unrounded) loss; Adam against torch.optim.Adam;
GELU against its definition; feature windows against direct indexing.
"""
import numpy as np
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
