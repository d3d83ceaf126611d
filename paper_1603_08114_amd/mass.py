"""Learned diagonal mass: binding of include/rsv_mlp.h and the training loop.

The network (27 -> 64 -> 64 -> 1, GELU, bfloat16 on the matrix cores) maps a
window of (ln y^2, ln RV) around each site and theta to log m_t.  Training
targets are -ln Var(h_t) measured from identity-mass chains: a diagonal mass
equal to the posterior precision equalises the scales the leapfrog sees.
Every arithmetic step (features, forward, backward, reduction, Adam) runs in
the HIP kernels; this module only marshals tensors and drives the loop.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .api import RSVError, lib

N_PARAMS = L.MLP_PARAMS
N_IN_PAD = L.MLP_INPUTS_PAD


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(st, where):
    if st != L.RSV_OK:
        raise RSVError(st, where)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def rsv_mlp_features(offsets_dev, y, log_rv, theta_series, mean, std, max_T, x, stream=None):
    n_series = offsets_dev.numel() - 1
    _check(lib().rsv_mlp_features(n_series, _p(offsets_dev), _p(y), _p(log_rv), _p(theta_series),
                                  _p(mean), _p(std), int(max_T), _p(x), _stream(stream)),
           "rsv_mlp_features")


def rsv_mlp_forward(x, params, out, clip=False, stream=None):
    _check(lib().rsv_mlp_forward(x.shape[0], _p(x), _p(params), _p(out), int(bool(clip)),
                                 _stream(stream)), "rsv_mlp_forward")


def rsv_mlp_grad(x, target, params, grad, loss, workspace, rows=None, n=None, stream=None):
    n = int(rows.numel() if rows is not None else x.shape[0]) if n is None else int(n)
    _check(lib().rsv_mlp_grad(n, _p(x), _p(target), _p(rows), _p(params), _p(grad), _p(loss),
                              _p(workspace), workspace.numel(), _stream(stream)), "rsv_mlp_grad")


def rsv_mlp_adam(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().rsv_mlp_adam(_p(params), _p(m), _p(v), _p(grad), int(step), float(lr),
                              float(beta1), float(beta2), float(eps), _stream(stream)),
           "rsv_mlp_adam")


def init_params(seed):
    """He initialisation of the flat FP32 parameter vector (layout of
    include/rsv_mlp.h); the input padding rows of W1 stay zero."""
    rng = np.random.default_rng(seed)
    n_in, n_pad, hid = L.MLP_INPUTS, L.MLP_INPUTS_PAD, L.MLP_HIDDEN
    w1 = np.zeros((n_pad, hid))
    w1[:n_in] = rng.standard_normal((n_in, hid)) * np.sqrt(2.0 / n_in)
    w2 = rng.standard_normal((hid, hid)) * np.sqrt(2.0 / hid)
    w3 = rng.standard_normal(hid) * np.sqrt(1.0 / hid)
    flat = np.concatenate([w1.ravel(), np.zeros(hid), w2.ravel(), np.zeros(hid), w3, [0.0]])
    assert flat.size == N_PARAMS
    return flat.astype(np.float32)


def grad_workspace(n, device="cuda"):
    nbytes = int(lib().rsv_mlp_grad_workspace_bytes(int(n)))
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


class MassNet:
    """FP32 master parameters on the device plus the input standardisation."""

    def __init__(self, params, mean, std, device="cuda"):
        self.device = torch.device(device)
        self.params = torch.as_tensor(np.asarray(params, np.float32), device=self.device).contiguous()
        assert self.params.numel() == N_PARAMS
        self.mean = torch.as_tensor(np.asarray(mean, np.float64), device=self.device).contiguous()
        self.std = torch.as_tensor(np.asarray(std, np.float64), device=self.device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0

    def features(self, offsets, y, log_rv, theta_series):
        """Inputs [n_sites, 32] (bfloat16 bit patterns in an int16 tensor)."""
        off = np.asarray(offsets, np.int64)
        off_d = torch.as_tensor(off, device=self.device)
        yd = torch.as_tensor(np.asarray(y, np.float64), device=self.device).contiguous()
        rd = torch.as_tensor(np.asarray(log_rv, np.float64), device=self.device).contiguous()
        th = torch.as_tensor(np.asarray(theta_series, np.float64).reshape(-1, 5),
                             device=self.device).contiguous()
        x = torch.empty((int(off[-1]), N_IN_PAD), dtype=torch.int16, device=self.device)
        rsv_mlp_features(off_d, yd, rd, th, self.mean, self.std, int(np.diff(off).max()), x)
        return x

    def forward(self, x, clip=False):
        out = torch.empty(x.shape[0], dtype=torch.float32, device=self.device)
        rsv_mlp_forward(x, self.params, out, clip)
        return out

    def gradient(self, x, target, rows=None):
        n = rows.numel() if rows is not None else x.shape[0]
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        rsv_mlp_grad(x, target, self.params, g, loss, grad_workspace(n, self.device), rows)
        return g, loss

    def fit(self, x, target, epochs, batch=8192, lr=2e-3, seed=0, log_every=0):
        """Adam on shuffled mini-batches; returns the mean loss of each epoch."""
        rng = np.random.default_rng(seed)
        n = x.shape[0]
        ws = grad_workspace(min(batch, n), self.device)
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        history = []
        for ep in range(epochs):
            perm = torch.as_tensor(rng.permutation(n).astype(np.int32), device=self.device)
            losses = []
            for s in range(0, n, batch):
                rows = perm[s:s + batch]
                rsv_mlp_grad(x, target, self.params, g, loss, ws, rows)
                self.step += 1
                rsv_mlp_adam(self.params, self.m, self.v, g, self.step, lr)
                losses.append(loss.clone())
            history.append(float(torch.cat(losses).mean().item()))
            if log_every and (ep + 1) % log_every == 0:
                print(f"[mass] epoch {ep + 1}: loss {history[-1]:.4f}", flush=True)
        return history

    def log_mass(self, x):
        return self.forward(x, clip=True)
