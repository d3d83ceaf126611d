"""ctypes front end of the FP64 CPU oracle (oracle/rsv_oracle.c).

TEST INFRASTRUCTURE ONLY.  The tests, ``__graft_entry__.smoke`` and the
benchmark's ``cpu_baseline`` leg may import this module; the product package
never does.  It shares no code with the HIP library.

Everything is plain numpy float64 in, float64 out.  ``theta`` is any mapping
with keys phi, mu, xi, sig2_eta, sig2_u (or a 5-sequence in that order).
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import build as _build

TERM_RETURN = 1
TERM_RV = 2
TERMS_RSV = 3
TAG_MOMENTUM, TAG_ACCEPT, TAG_THETA = 0, 1, 2
THETA_KEYS = ("phi", "mu", "xi", "sig2_eta", "sig2_u")
PRIOR_KEYS = ("mu_mean", "mu_var", "xi_mean", "xi_var",
              "eta_shape", "eta_scale", "u_shape", "u_scale")
# Priors of the theta update (readings; the paper gives none).
DEFAULT_PRIOR = dict(mu_mean=0.0, mu_var=100.0, xi_mean=0.0, xi_var=100.0,
                     eta_shape=1.0, eta_scale=0.01, u_shape=1.0, u_scale=0.01)


class Theta(C.Structure):
    _fields_ = [(k, C.c_double) for k in THETA_KEYS]

    def as_dict(self):
        return {k: getattr(self, k) for k in THETA_KEYS}


class Prior(C.Structure):
    _fields_ = [(k, C.c_double) for k in PRIOR_KEYS]


_D = C.POINTER(C.c_double)
_U64 = C.c_uint64
_I64 = C.c_int64


def _load():
    if not _build.up_to_date():
        _build.build()
    lib = C.CDLL(_build.LIB)
    P = C.POINTER
    sig = {
        "orc_philox4x64_10": (None, [P(_U64), P(_U64), P(_U64)]),
        "orc_uniforms4": (None, [_U64, _U64, _U64, _U64, _U64, _D]),
        "orc_uniform_stream": (None, [_U64, _U64, _U64, _U64, _I64, _D]),
        "orc_normal_stream": (None, [_U64, _U64, _U64, _U64, _I64, _D]),
        "orc_energy": (C.c_double, [_I64, _D, _D, _D, P(Theta), C.c_int]),
        "orc_grad": (None, [_I64, _D, _D, _D, P(Theta), C.c_int, _D]),
        "orc_hamiltonian": (C.c_double, [_I64, _D, _D, _D, _D, _D, P(Theta), C.c_int]),
        "orc_leapfrog": (None, [_I64, _D, _D, _D, _D, _D, P(Theta), C.c_int, C.c_int32,
                                C.c_double]),
        "orc_omelyan": (None, [_I64, _D, _D, _D, _D, _D, P(Theta), C.c_int, C.c_int32,
                               C.c_double]),
        "orc_forest_ruth": (None, [_I64, _D, _D, _D, _D, _D, P(Theta), C.c_int, C.c_int32,
                                   C.c_double]),
        "orc_delta_h": (C.c_double, [_I64, _D, _D, _D, _D, _D, _D, _D, P(Theta), C.c_int]),
        "orc_momenta": (None, [_U64, _U64, _U64, _I64, _D, _D]),
        "orc_momenta_f32": (None, [_U64, _U64, _U64, _I64, _D, _D]),
        "orc_log_u": (C.c_double, [_U64, _U64, _U64]),
        "orc_trajectory": (C.c_int, [_I64, _D, _D, _D, _D, P(Theta), C.c_int, C.c_int32,
                                     C.c_double, C.c_int, _U64, _U64, _U64, _D, _D, _D, _D]),
        "orc_suffstats": (None, [_I64, _D, _D, C.c_double, C.c_double, _D]),
        "orc_theta_update": (C.c_int, [_I64, _D, P(Theta), P(Prior), C.c_int, _U64, _U64,
                                       _U64, P(Theta)]),
        "orc_draw_mu": (C.c_double, [_I64, _D, P(Theta), P(Prior), C.c_double]),
        "orc_draw_xi": (C.c_double, [_I64, _D, P(Theta), P(Prior), C.c_double]),
        "orc_gamma": (C.c_double, [C.c_double, _U64, _U64, _U64, _U64, _U64,
                                   P(C.c_int)]),
        "orc_neumaier_sum": (C.c_double, [_I64, _D]),
        "orc_step_size": (C.c_double, [_U64, _U64, _U64, C.c_double, C.c_double]),
        "orc_level_move": (C.c_int, [_I64, _D, P(Theta), _D, P(Prior), C.c_int, _U64, _U64,
                                     _U64, _D]),
        "orc_run": (_I64, [_I64, _D, P(Theta), _D, _D, _D, P(Prior), C.c_int, C.c_int32,
                           C.c_double, C.c_double, C.c_int, C.c_int, _U64, _U64, _U64, _I64,
                           C.c_int, _D,
                           P(C.c_int32), P(Theta), _D]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def _arr(x, n=None):
    a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def theta_struct(theta) -> Theta:
    if isinstance(theta, Theta):
        return theta
    if isinstance(theta, dict):
        return Theta(*[float(theta[k]) for k in THETA_KEYS])
    return Theta(*[float(v) for v in theta])


def prior_struct(prior=None) -> Prior:
    p = dict(DEFAULT_PRIOR)
    if prior:
        p.update(prior)
    return Prior(*[float(p[k]) for k in PRIOR_KEYS])


# --- random numbers ---------------------------------------------------------
def philox4x64_10(ctr, key):
    c = (_U64 * 4)(*[int(v) for v in ctr])
    k = (_U64 * 2)(*[int(v) for v in key])
    out = (_U64 * 4)()
    _lib.orc_philox4x64_10(c, k, out)
    return np.array(list(out), dtype=np.uint64)


def uniforms4(seed, idx, sweep, chain, tag):
    u = np.zeros(4)
    _lib.orc_uniforms4(seed, idx, sweep, chain, tag, _ptr(u))
    return u


def uniform_stream(seed, sweep, chain, tag, n):
    out = np.zeros(n)
    _lib.orc_uniform_stream(seed, sweep, chain, tag, n, _ptr(out))
    return out


def normal_stream(seed, sweep, chain, tag, n):
    out = np.zeros(n)
    _lib.orc_normal_stream(seed, sweep, chain, tag, n, _ptr(out))
    return out


# --- target, force, integrator ----------------------------------------------
def energy(h, y2, r, theta, terms=TERMS_RSV):
    h = _arr(h); T = h.size
    return _lib.orc_energy(T, _ptr(h), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                           C.byref(theta_struct(theta)), terms)


def grad(h, y2, r, theta, terms=TERMS_RSV):
    h = _arr(h); T = h.size
    g = np.zeros(T)
    _lib.orc_grad(T, _ptr(h), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                  C.byref(theta_struct(theta)), terms, _ptr(g))
    return g


def hamiltonian(h, p, y2, r, theta, terms=TERMS_RSV, log_m=None):
    h = _arr(h); T = h.size
    lm = None if log_m is None else _arr(log_m, T)
    return _lib.orc_hamiltonian(T, _ptr(h), _ptr(_arr(p, T)), _ptr(lm), _ptr(_arr(y2, T)),
                                _ptr(_arr(r, T)), C.byref(theta_struct(theta)), terms)


def leapfrog(h, p, y2, r, theta, k, dtau, terms=TERMS_RSV, log_m=None):
    """k steps of eqs. (6)-(8); returns new (h, p) (inputs untouched)."""
    h = _arr(h).copy(); T = h.size
    p = _arr(p, T).copy()
    lm = None if log_m is None else _arr(log_m, T)
    _lib.orc_leapfrog(T, _ptr(h), _ptr(p), _ptr(lm), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                      C.byref(theta_struct(theta)), terms, int(k), float(dtau))
    return h, p


INT_LEAPFROG = 0
INT_OMELYAN = 1
INT_FOREST_RUTH = 2
OMELYAN_LAMBDA = 0.1931833275037836
FOREST_RUTH_THETA = 1.3512071919596578


def omelyan(h, p, y2, r, theta, k, dtau, terms=TERMS_RSV, log_m=None):
    """k steps of Omelyan's second-order minimum-norm scheme (h first);
    returns new (h, p) (inputs untouched)."""
    h = _arr(h).copy(); T = h.size
    p = _arr(p, T).copy()
    lm = None if log_m is None else _arr(log_m, T)
    _lib.orc_omelyan(T, _ptr(h), _ptr(p), _ptr(lm), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                     C.byref(theta_struct(theta)), terms, int(k), float(dtau))
    return h, p


def forest_ruth(h, p, y2, r, theta, k, dtau, terms=TERMS_RSV, log_m=None):
    """k steps of Forest and Ruth's fourth-order scheme (h first); returns
    new (h, p) (inputs untouched)."""
    h = _arr(h).copy(); T = h.size
    p = _arr(p, T).copy()
    lm = None if log_m is None else _arr(log_m, T)
    _lib.orc_forest_ruth(T, _ptr(h), _ptr(p), _ptr(lm), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                         C.byref(theta_struct(theta)), terms, int(k), float(dtau))
    return h, p


def delta_h(h0, p0, h1, p1, y2, r, theta, terms=TERMS_RSV, log_m=None):
    h0 = _arr(h0); T = h0.size
    lm = None if log_m is None else _arr(log_m, T)
    return _lib.orc_delta_h(T, _ptr(h0), _ptr(_arr(p0, T)), _ptr(_arr(h1, T)),
                            _ptr(_arr(p1, T)), _ptr(lm), _ptr(_arr(y2, T)),
                            _ptr(_arr(r, T)), C.byref(theta_struct(theta)), terms)


def momenta(seed, sweep, chain, T, log_m=None):
    p = np.zeros(T)
    lm = None if log_m is None else _arr(log_m, T)
    _lib.orc_momenta(seed, sweep, chain, T, _ptr(lm), _ptr(p))
    return p


def momenta_f32(seed, sweep, chain, T, log_m=None):
    """Momenta of the FP32-mixed path's stream layout, in FP64."""
    p = np.zeros(T)
    lm = None if log_m is None else _arr(log_m, T)
    _lib.orc_momenta_f32(seed, sweep, chain, T, _ptr(lm), _ptr(p))
    return p


def log_u(seed, sweep, chain):
    return _lib.orc_log_u(seed, sweep, chain)


def step_size(seed, sweep, chain, dtau, jitter):
    """dtau of (seed, sweep, chain) under step-size jitter (jitter 0: dtau)."""
    return _lib.orc_step_size(seed, sweep, chain, float(dtau), float(jitter))


def trajectory(h, y2, r, theta, k, dtau, seed=0, sweep=0, chain=0, terms=TERMS_RSV,
               p0=None, log_u=None, log_m=None, jitter=0.0, integrator=INT_LEAPFROG):
    """One HMC trajectory.  Returns dict(h, accepted, dH, p0)."""
    dtau = step_size(seed, sweep, chain, dtau, jitter)
    h = _arr(h).copy(); T = h.size
    lm = None if log_m is None else _arr(log_m, T)
    p0a = None if p0 is None else _arr(p0, T)
    lu = None if log_u is None else np.array([float(log_u)])
    p_used = np.zeros(T)
    dH = np.zeros(1)
    acc = _lib.orc_trajectory(T, _ptr(h), _ptr(lm), _ptr(_arr(y2, T)), _ptr(_arr(r, T)),
                              C.byref(theta_struct(theta)), terms, int(k), float(dtau),
                              int(integrator), seed, sweep, chain, _ptr(p0a), _ptr(lu),
                              _ptr(p_used), _ptr(dH))
    return dict(h=h, accepted=bool(acc), dH=float(dH[0]), p0=p_used)


# --- theta update ------------------------------------------------------------
def suffstats(h, r, c_mu, c_xi):
    h = _arr(h); T = h.size
    out = np.zeros(7)
    _lib.orc_suffstats(T, _ptr(h), _ptr(_arr(r, T)), float(c_mu), float(c_xi), _ptr(out))
    return out


def theta_update(T, stats, theta, seed, sweep, chain, prior=None, terms=TERMS_RSV):
    """Returns (new theta dict, flags)."""
    out = Theta()
    flags = _lib.orc_theta_update(int(T), _ptr(_arr(stats, 7)), C.byref(theta_struct(theta)),
                                  C.byref(prior_struct(prior)), terms, seed, sweep, chain,
                                  C.byref(out))
    return out.as_dict(), flags


MOVE_LEVEL = 2
TAG_MOVE = 4


def level_move(h, theta, y2, seed, sweep, chain, prior=None, terms=TERMS_RSV):
    """The level move on (h, theta).  Returns dict(h, theta, flags, c)."""
    h = _arr(h).copy(); T = h.size
    th = theta_struct(theta)
    th = Theta(*[getattr(th, k_) for k_ in THETA_KEYS])
    c_out = np.zeros(1)
    flags = _lib.orc_level_move(T, _ptr(h), C.byref(th), _ptr(_arr(y2, T)),
                                C.byref(prior_struct(prior)), terms, seed, sweep, chain,
                                _ptr(c_out))
    return dict(h=h, theta=th.as_dict(), flags=flags, c=float(c_out[0]))


def draw_mu(T, stats, theta, z, prior=None):
    return _lib.orc_draw_mu(int(T), _ptr(_arr(stats, 7)), C.byref(theta_struct(theta)),
                            C.byref(prior_struct(prior)), float(z))


def draw_xi(T, stats, theta, z, prior=None):
    return _lib.orc_draw_xi(int(T), _ptr(_arr(stats, 7)), C.byref(theta_struct(theta)),
                            C.byref(prior_struct(prior)), float(z))


def gamma(alpha, seed, sweep, chain, tag=TAG_THETA, idx0=2):
    ex = C.c_int(0)
    v = _lib.orc_gamma(float(alpha), seed, sweep, chain, tag, idx0, C.byref(ex))
    return v, bool(ex.value)


def neumaier_sum(x):
    x = _arr(x)
    return _lib.orc_neumaier_sum(x.size, _ptr(x))


def run(h, theta, y2, r, k, dtau, n_sweeps, seed=0, chain=0, first_sweep=0,
        update_theta=True, prior=None, terms=TERMS_RSV, log_m=None, keep_h=False, jitter=0.0,
        moves=0, integrator=INT_LEAPFROG):
    """n sweeps of one chain.  Returns dict with final h/theta and traces."""
    h = _arr(h).copy(); T = h.size
    th = theta_struct(theta)
    th = Theta(*[getattr(th, k_) for k_ in THETA_KEYS])
    lm = None if log_m is None else _arr(log_m, T)
    dH = np.zeros(n_sweeps)
    acc = np.zeros(n_sweeps, dtype=np.int32)
    ttrace = (Theta * n_sweeps)()
    htrace = np.zeros((n_sweeps, T)) if keep_h else None
    n_acc = _lib.orc_run(T, _ptr(h), C.byref(th), _ptr(lm), _ptr(_arr(y2, T)),
                         _ptr(_arr(r, T)), C.byref(prior_struct(prior)), terms, int(k),
                         float(dtau), float(jitter), int(moves), int(integrator), seed, chain,
                         first_sweep,
                         n_sweeps, int(update_theta),
                         _ptr(dH), acc.ctypes.data_as(C.POINTER(C.c_int32)), ttrace,
                         _ptr(htrace))
    theta_tr = np.array([[getattr(ttrace[i], k_) for k_ in THETA_KEYS]
                         for i in range(n_sweeps)])
    return dict(h=h, theta=th.as_dict(), dH=dH, accepted=acc.astype(bool),
                theta_trace=theta_tr, h_trace=htrace, n_accepted=int(n_acc))


LIB_PATH = _build.LIB
