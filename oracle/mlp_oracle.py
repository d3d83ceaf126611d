"""FP64 oracle of the learned diagonal-mass network (test infrastructure only).

A 27 -> 64 -> 64 -> 1 perceptron with GELU (exact erf form) maps, for each
site t of a series, an 11-site window of (ln y^2, ln RV) and the series'
theta to log m_t, the log of the diagonal mass of the HMC kinetic energy
(H = sum p^2/(2 m) + U, a preconditioned form of the Hamiltonian of Sec. 3;
the paper itself uses m = 1).  The target of training is -ln Var(h_t), the
log posterior precision of each site estimated from plain chains.

Rounding points of the GPU kernels are emulated when ``bf16=True``:
inputs, weights and hidden activations rounded to bfloat16 (round to
nearest even); products accumulated, biases added and GELU taken in wide
precision.  With ``bf16=False`` everything is FP64 (used for the
finite-difference check of the gradients).

Only tests, the smoke check and the benchmark's CPU leg use this module.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

WINDOW = 5                      # sites on each side of t
N_IN = 2 * (2 * WINDOW + 1) + 5  # 27
N_IN_PAD = 32
HIDDEN = 64
THETA_KEYS = ("phi", "mu", "xi", "sig2_eta", "sig2_u")
LOG_MASS_CLIP = 5.0
Y2_FLOOR = 1e-8


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return rounded.view(np.float32).astype(np.float64)


def raw_features(y2, log_rv, theta):
    """Unstandardised inputs [T, 27] of one series: ln(y^2 + floor) and ln RV
    at t-5..t+5 (indices clamped to the series), then theta."""
    T = len(y2)
    idx = np.clip(np.arange(T)[:, None] + np.arange(-WINDOW, WINDOW + 1)[None, :], 0, T - 1)
    ly = np.log(np.asarray(y2, np.float64) + Y2_FLOOR)
    lr = np.asarray(log_rv, np.float64)
    th = np.array([theta[k] for k in THETA_KEYS], np.float64)
    return np.concatenate([ly[idx], lr[idx], np.broadcast_to(th, (T, 5))], axis=1)


def standardise(raw, mean, std):
    return (raw - mean) / std


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def init_params(seed):
    """He-style initialisation; W1 rows 27..31 (input padding) are zero."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((N_IN_PAD, HIDDEN))
    W1[:N_IN] = rng.standard_normal((N_IN, HIDDEN)) * np.sqrt(2.0 / N_IN)
    return dict(W1=W1, b1=np.zeros(HIDDEN),
                W2=rng.standard_normal((HIDDEN, HIDDEN)) * np.sqrt(2.0 / HIDDEN),
                b2=np.zeros(HIDDEN),
                w3=rng.standard_normal(HIDDEN) * np.sqrt(1.0 / HIDDEN), b3=np.zeros(1))


PARAM_SHAPES = (("W1", (N_IN_PAD, HIDDEN)), ("b1", (HIDDEN,)), ("W2", (HIDDEN, HIDDEN)),
                ("b2", (HIDDEN,)), ("w3", (HIDDEN,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def flatten(p):
    return np.concatenate([np.asarray(p[k], np.float64).ravel() for k, _ in PARAM_SHAPES])


def unflatten(v):
    out, i = {}, 0
    for k, s in PARAM_SHAPES:
        n = int(np.prod(s))
        out[k] = np.asarray(v[i:i + n], np.float64).reshape(s)
        i += n
    return out


def forward(p, X, bf16=True):
    """X [n, 32] standardised inputs (padding columns zero).  Returns the
    output [n] and the intermediate values the backward pass needs."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    x = r(X)
    W1, W2, w3 = r(p["W1"]), r(p["W2"]), r(p["w3"])
    pre1 = x @ W1 + p["b1"]
    h1 = r(gelu(pre1))
    pre2 = h1 @ W2 + p["b2"]
    h2 = r(gelu(pre2))
    out = h2 @ w3 + p["b3"][0]
    return out, dict(x=x, W1=W1, W2=W2, w3=w3, pre1=pre1, h1=h1, pre2=pre2, h2=h2)


def loss(p, X, target, bf16=True):
    out, _ = forward(p, X, bf16)
    return float(np.mean((out - target) ** 2))


def grad(p, X, target, bf16=True):
    """Gradient of the mean squared error; with bf16=True the back-propagated
    signals are rounded where the GPU rounds them (before each product)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    out, c = forward(p, X, bf16)
    n = X.shape[0]
    dout = 2.0 * (out - target) / n
    dpre2 = np.outer(dout, c["w3"]) * gelu_grad(c["pre2"])
    dpre2_r = r(dpre2)
    dW2 = c["h1"].T @ dpre2_r
    dh1 = dpre2_r @ c["W2"].T
    dpre1 = dh1 * gelu_grad(c["pre1"])
    dW1 = c["x"].T @ r(dpre1)
    return dict(W1=dW1, b1=dpre1.sum(0), W2=dW2, b2=dpre2.sum(0),
                w3=c["h2"].T @ dout, b3=np.array([dout.sum()]))


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) on every array of p, in place."""
    for k in p:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] * g[k]
        mh = m[k] / (1 - b1 ** step)
        vh = v[k] / (1 - b2 ** step)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def log_mass(p, X, bf16=True):
    """The network output clipped to [-5, 5] where finite; a non-finite
    output is returned as it is (the sampler's identity fallback handles it)."""
    out, _ = forward(p, X, bf16)
    return np.where(np.isfinite(out), np.clip(out, -LOG_MASS_CLIP, LOG_MASS_CLIP), out)
