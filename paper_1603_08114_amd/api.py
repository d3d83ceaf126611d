"""Python binding of the RSV HMC library: argument marshalling only.

Functions carry the C names of include/rsv_hmc.h and take torch tensors for
device memory (PyTorch owns every allocation and the stream); every step of
the sampler runs in the HIP kernels of librsvhmc.so.  ``RSVSampler`` bundles
the tensors one context needs.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = L.load()
    return _lib


class RSVError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = lib().rsv_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status: int, where: str):
    if status != L.RSV_OK:
        raise RSVError(status, where)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


DEFAULT_PRIOR = dict(mu_mean=0.0, mu_var=100.0, xi_mean=0.0, xi_var=100.0,
                     eta_shape=1.0, eta_scale=0.01, u_shape=1.0, u_scale=0.01)


@dataclass
class Problem:
    """Host description of the series; y and log_rv are FP64 device tensors."""
    offsets: np.ndarray
    y: torch.Tensor
    log_rv: torch.Tensor
    chains_per_series: int = 1
    precision: int = L.RSV_F64
    terms: int = L.RSV_TERMS_RSV
    max_steps: int = 50
    sites_per_lane: int = 0
    waves_per_tile: int = 0
    flags: int = 0
    seed: int = 0
    dtau_jitter: float = 0.0
    prior: dict = field(default_factory=lambda: dict(DEFAULT_PRIOR))

    def __post_init__(self):
        self.offsets = np.ascontiguousarray(self.offsets, dtype=np.int64)

    @property
    def n_series(self):
        return int(self.offsets.size - 1)

    @property
    def n_chains(self):
        return self.n_series * self.chains_per_series

    def struct(self) -> L.rsv_problem:
        pb = L.rsv_problem()
        pb.n_series = self.n_series
        pb.chains_per_series = int(self.chains_per_series)
        pb.offsets = self.offsets.ctypes.data_as(C.POINTER(C.c_int64))
        pb.y = _ptr(self.y).value if self.y is not None else None
        pb.log_rv = _ptr(self.log_rv).value if self.log_rv is not None else None
        pb.precision = int(self.precision)
        pb.terms = int(self.terms)
        pb.max_steps = int(self.max_steps)
        pb.sites_per_lane = int(self.sites_per_lane)
        pb.waves_per_tile = int(self.waves_per_tile)
        pb.flags = int(self.flags)
        pb.seed = int(self.seed)
        pb.dtau_jitter = float(self.dtau_jitter)
        pr = dict(DEFAULT_PRIOR)
        pr.update(self.prior or {})
        pb.prior = L.rsv_prior(*[float(pr[k]) for k in L.PRIOR_KEYS])
        self._keep = pb  # the offsets pointer must stay valid
        return pb


def leapfrog_array(lf, n_series: int):
    """(k, dtau) or a list of them -> ctypes array of rsv_leapfrog, one per series."""
    if isinstance(lf, tuple) and len(lf) == 2 and not isinstance(lf[0], (tuple, list)):
        lf = [lf] * n_series
    arr = (L.rsv_leapfrog * n_series)()
    for s, (k, dt) in enumerate(lf):
        arr[s].n_steps = int(k)
        arr[s].reserved = 0
        arr[s].dtau = float(dt)
    return arr


# --- the C entry points -------------------------------------------------------
def rsv_hmc_workspace_bytes(pb: Problem) -> int:
    n = lib().rsv_hmc_workspace_bytes(C.byref(pb.struct()))
    if n == 0:
        raise RSVError(L.RSV_EINVAL, "rsv_hmc_workspace_bytes")
    return int(n)


def rsv_hmc_state_size(pb: Problem) -> int:
    return int(lib().rsv_hmc_state_size(C.byref(pb.struct())))


def rsv_hmc_init(pb: Problem, h: torch.Tensor, theta: torch.Tensor,
                 log_mass: Optional[torch.Tensor], workspace: torch.Tensor,
                 stream: Optional[torch.cuda.Stream] = None) -> C.c_void_p:
    ctx = C.c_void_p()
    st = lib().rsv_hmc_init(C.byref(ctx), C.byref(pb.struct()), _ptr(h), _ptr(theta),
                            _ptr(log_mass), _ptr(workspace), workspace.numel(),
                            _stream_handle(stream))
    _check(st, "rsv_hmc_init")
    return ctx


def rsv_hmc_init_static(pb: Problem, h: torch.Tensor, theta: torch.Tensor,
                        log_mass: Optional[torch.Tensor],
                        stream: Optional[torch.cuda.Stream] = None) -> C.c_void_p:
    ctx = C.c_void_p()
    st = lib().rsv_hmc_init_static(C.byref(ctx), C.byref(pb.struct()), _ptr(h), _ptr(theta),
                                   _ptr(log_mass), _stream_handle(stream))
    _check(st, "rsv_hmc_init_static")
    return ctx


def rsv_hmc_momenta(ctx, sweep: int, p_out: torch.Tensor):
    _check(lib().rsv_hmc_momenta(ctx, int(sweep), _ptr(p_out)), "rsv_hmc_momenta")


def rsv_hmc_trajectory(ctx, sweep: int, lf, p0=None, log_u=None, delta_h=None,
                       accepted=None):
    _check(lib().rsv_hmc_trajectory(ctx, int(sweep), lf, _ptr(p0), _ptr(log_u),
                                    _ptr(delta_h), _ptr(accepted)), "rsv_hmc_trajectory")


def rsv_theta_update(ctx, sweep: int, suff_stats=None):
    _check(lib().rsv_theta_update(ctx, int(sweep), _ptr(suff_stats)), "rsv_theta_update")


def rsv_hmc_sweep(ctx, first_sweep: int, n_sweeps: int, lf, update_theta: bool,
                  trace: Optional[L.rsv_trace] = None):
    _check(lib().rsv_hmc_sweep(ctx, int(first_sweep), int(n_sweeps), lf, int(bool(update_theta)),
                               C.byref(trace) if trace is not None else None),
           "rsv_hmc_sweep")


def rsv_hmc_check(ctx):
    n = C.c_int64(0)
    st = lib().rsv_hmc_check(ctx, C.byref(n))
    return int(st), int(n.value)


def rsv_hmc_profile(ctx, max_records: int):
    _check(lib().rsv_hmc_profile(ctx, int(max_records)), "rsv_hmc_profile")


def rsv_hmc_kernel_time(ctx):
    """(summed milliseconds, number of records) of the recorded trajectories."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(lib().rsv_hmc_kernel_time(ctx, C.byref(ms), C.byref(n)), "rsv_hmc_kernel_time")
    return float(ms.value), int(n.value)


def rsv_hmc_destroy(ctx):
    _check(lib().rsv_hmc_destroy(ctx), "rsv_hmc_destroy")


# --- convenience owner of one context's tensors --------------------------------
def theta_tensor(thetas, n_chains: int, device) -> torch.Tensor:
    """dict / list of dicts / [n,5] array -> [n_chains, 5] FP64 device tensor."""
    if isinstance(thetas, dict):
        arr = np.array([[thetas[k] for k in L.THETA_KEYS]] * n_chains, dtype=np.float64)
    else:
        arr = np.asarray([[t[k] for k in L.THETA_KEYS] if isinstance(t, dict) else list(t)
                          for t in thetas], dtype=np.float64)
    if arr.shape != (n_chains, 5):
        raise ValueError(f"theta must give {n_chains} chains, got shape {arr.shape}")
    return torch.tensor(arr, dtype=torch.float64, device=device)


class RSVSampler:
    """Tensors + context for one problem.  ``h`` holds every chain's state in
    the layout of include/rsv_hmc.h; ``theta`` is [n_chains, 5]."""

    def __init__(self, offsets, y, log_rv, h0, theta0, chains_per_series=1,
                 precision=L.RSV_F64, terms=L.RSV_TERMS_RSV, max_steps=50, seed=0,
                 prior=None, log_mass=None, sites_per_lane=0, waves_per_tile=0, flags=0,
                 dtau_jitter=0.0, device="cuda", static_workspace=False):
        if not torch.cuda.is_available():
            raise RuntimeError("RSVSampler needs a GPU (HIP device)")
        self.device = torch.device(device)
        to = dict(device=self.device)
        self.y = torch.as_tensor(np.asarray(y, np.float64), **to).contiguous()
        self.log_rv = torch.as_tensor(np.asarray(log_rv, np.float64), **to).contiguous()
        self.pb = Problem(offsets=np.asarray(offsets, np.int64), y=self.y, log_rv=self.log_rv,
                          chains_per_series=chains_per_series, precision=precision, terms=terms,
                          max_steps=max_steps, sites_per_lane=sites_per_lane,
                          waves_per_tile=waves_per_tile, flags=flags, seed=seed,
                          dtau_jitter=dtau_jitter, prior=prior or dict(DEFAULT_PRIOR))
        state_dtype = torch.float64 if precision == L.RSV_F64 else torch.float32
        self.n_state = rsv_hmc_state_size(self.pb)
        self.h = torch.as_tensor(np.asarray(h0, np.float64), **to).to(state_dtype).contiguous()
        if self.h.numel() != self.n_state:
            raise ValueError(f"h0 has {self.h.numel()} entries, the problem needs {self.n_state}")
        self.theta = theta_tensor(theta0, self.pb.n_chains, self.device).contiguous()
        self.log_mass = None
        if log_mass is not None:
            self.log_mass = torch.as_tensor(np.asarray(log_mass, np.float32), **to).contiguous()
        self.stream = torch.cuda.current_stream(self.device)
        if static_workspace:  # the library's own device array (rsv_hmc_init_static)
            self.workspace = None
            self.ctx = rsv_hmc_init_static(self.pb, self.h, self.theta, self.log_mass,
                                           self.stream)
            return
        nbytes = rsv_hmc_workspace_bytes(self.pb)
        # 256-byte aligned workspace carved from a uint8 tensor
        self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        shift = (-self._ws_raw.data_ptr()) % 256
        self.workspace = self._ws_raw[shift:shift + nbytes]
        self.ctx = rsv_hmc_init(self.pb, self.h, self.theta, self.log_mass, self.workspace,
                                self.stream)

    @property
    def n_chains(self):
        return self.pb.n_chains

    def leapfrog(self, lf):
        return leapfrog_array(lf, self.pb.n_series)

    def momenta(self, sweep):
        p = torch.empty(self.n_state, dtype=torch.float64, device=self.device)
        rsv_hmc_momenta(self.ctx, sweep, p)
        return p

    def trajectory(self, sweep, lf, p0=None, log_u=None):
        dh = torch.empty(self.n_chains, dtype=torch.float64, device=self.device)
        acc = torch.empty(self.n_chains, dtype=torch.int32, device=self.device)
        p0t = None if p0 is None else torch.as_tensor(p0, dtype=torch.float64,
                                                      device=self.device).contiguous()
        lut = None if log_u is None else torch.as_tensor(log_u, dtype=torch.float64,
                                                         device=self.device).reshape(-1).contiguous()
        rsv_hmc_trajectory(self.ctx, sweep, self.leapfrog(lf), p0t, lut, dh, acc)
        return dh, acc

    def theta_update(self, sweep, want_stats=True):
        st = torch.empty((self.n_chains, 7), dtype=torch.float64, device=self.device) \
            if want_stats else None
        rsv_theta_update(self.ctx, sweep, st)
        return st

    def sweep(self, first_sweep, n_sweeps, lf, update_theta=True, record=("delta_h", "accepted",
                                                                              "theta"),
              record_h=False, batch_len=0):
        """n sweeps; ``record`` names per-sweep traces to return, ``record_h``
        stores h after every sweep, ``batch_len`` > 0 accumulates batch sums of
        h (and the sum of h^2) on the device instead."""
        n, nc = int(n_sweeps), self.n_chains
        out = {}
        tr = L.rsv_trace()
        if batch_len:
            nb = (n + batch_len - 1) // batch_len
            out["h_batch_sum"] = torch.zeros((nb, self.n_state), dtype=torch.float64,
                                             device=self.device)
            out["h_sq_sum"] = torch.zeros(self.n_state, dtype=torch.float64, device=self.device)
            tr.h_batch_sum = out["h_batch_sum"].data_ptr()
            tr.h_sq_sum = out["h_sq_sum"].data_ptr()
            tr.batch_len = int(batch_len)
        if "delta_h" in record:
            out["delta_h"] = torch.empty((n, nc), dtype=torch.float64, device=self.device)
            tr.delta_h = out["delta_h"].data_ptr()
        if "accepted" in record:
            out["accepted"] = torch.empty((n, nc), dtype=torch.int32, device=self.device)
            tr.accepted = out["accepted"].data_ptr()
        if "theta" in record:
            out["theta"] = torch.empty((n, nc, 5), dtype=torch.float64, device=self.device)
            tr.theta = out["theta"].data_ptr()
        if record_h:
            out["h"] = torch.empty((n, self.n_state), dtype=self.h.dtype, device=self.device)
            tr.h = out["h"].data_ptr()
        rsv_hmc_sweep(self.ctx, first_sweep, n, self.leapfrog(lf), update_theta,
                      tr if out else None)
        return out

    def check(self):
        return rsv_hmc_check(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            rsv_hmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
