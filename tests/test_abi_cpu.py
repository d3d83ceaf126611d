"""The C-ABI library loads without a GPU, exports every symbol its header
declares, and rejects invalid problems on the host before any device call."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1603_08114_amd import _lib, api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rsv_\w+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("rsv_hmc_init", "rsv_hmc_trajectory", "rsv_hmc_sweep", "rsv_theta_update"):
        assert required in names
    assert sorted(_lib.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(_lib.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_struct_sizes_match_header_layout():
    assert C.sizeof(_lib.rsv_theta) == 40
    assert C.sizeof(_lib.rsv_prior) == 64
    assert C.sizeof(_lib.rsv_leapfrog) == 16
    assert C.sizeof(_lib.rsv_problem) == 4 + 4 + 8 * 3 + 4 * 6 + 8 + 8 + 64
    assert C.sizeof(_lib.rsv_trace) == 56


def _pb(offsets, **kw):
    return api.Problem(offsets=np.asarray(offsets), y=None, log_rv=None, **kw)


def test_workspace_and_state_sizes():
    pb = _pb([0, 1000, 5000], chains_per_series=4, max_steps=30)
    assert api.rsv_hmc_state_size(pb) == 4 * 5000
    n64 = api.rsv_hmc_workspace_bytes(pb)
    pb32 = _pb([0, 1000, 5000], chains_per_series=4, max_steps=30, precision=_lib.RSV_F32_MIXED)
    assert n64 > 0 and api.rsv_hmc_workspace_bytes(pb32) > 0
    # the proposal buffer alone is n_state * 8 bytes in FP64
    assert n64 >= 4 * 5000 * 8


@pytest.mark.parametrize("bad", [
    dict(offsets=[0, 2]),                         # T < 3
    dict(offsets=[1, 5]),                         # offsets[0] != 0
    dict(offsets=[0, 100], max_steps=0),
    dict(offsets=[0, 100], precision=7),
    dict(offsets=[0, 100], terms=0),
    dict(offsets=[0, 100], sites_per_lane=5),
    dict(offsets=[0, 100], chains_per_series=0),
    dict(offsets=[0, 5000], max_steps=400, sites_per_lane=8, waves_per_tile=1),  # halo > tile
    dict(offsets=[0, 100], waves_per_tile=3),
    dict(offsets=[0, 100], dtau_jitter=1.0),
    dict(offsets=[0, 100], dtau_jitter=-0.1),
    dict(offsets=[0, 100], flags=16),                                  # unknown flag
    dict(offsets=[0, 100], flags=4 | 8),                               # two integrators
    dict(offsets=[0, 3000], max_steps=50, sites_per_lane=4, waves_per_tile=1,
         flags=8),                                                    # 3k-kick halo > tile
    dict(offsets=[0, 100], prior=dict(mu_var=-1.0)),
])
def test_invalid_problems_rejected_on_host(bad):
    offsets = bad.pop("offsets")
    pb = _pb(offsets, **bad)
    with pytest.raises(api.RSVError) as e:
        api.rsv_hmc_workspace_bytes(pb)
    assert e.value.status == _lib.RSV_EINVAL
    assert len(_lib.load().rsv_last_error()) > 0
    # init fails the same way, before touching a device
    ctx = C.c_void_p()
    st = _lib.load().rsv_hmc_init(C.byref(ctx), C.byref(pb.struct()), None, None, None, None,
                                  0, None)
    assert st == _lib.RSV_EINVAL and not ctx.value


def test_mlp_host_validation():
    lib = _lib.load()
    assert lib.rsv_mlp_grad_workspace_bytes(0) == 0
    assert lib.rsv_mlp_grad_workspace_bytes(65) == 2 * (_lib.MLP_PARAMS + 1) * 4
    assert lib.rsv_mlp_forward(0, None, None, None, 0, None) == _lib.RSV_EINVAL
    assert lib.rsv_mlp_grad(10, None, None, None, None, None, None, None, 0, None) == _lib.RSV_EINVAL
    assert lib.rsv_mlp_adam(None, None, None, None, 1, 1e-3, 0.9, 0.999, 1e-8, None) == _lib.RSV_EINVAL
    assert b"rsv_mlp_adam" in lib.rsv_last_error()


def test_null_context_is_a_state_error():
    lib = _lib.load()
    lf = (_lib.rsv_leapfrog * 1)()
    assert lib.rsv_hmc_trajectory(None, 0, lf, None, None, None, None) == _lib.RSV_ESTATE
    assert lib.rsv_theta_update(None, 0, None) == _lib.RSV_ESTATE
    assert lib.rsv_hmc_sweep(None, 0, 1, lf, 1, None) == _lib.RSV_ESTATE


def test_autotune_cache_key_buckets():
    """Host logic of the tile-shape autotuner: problems in one (precision, k,
    T bucket, chain-count bucket) share a cache entry."""
    from paper_1603_08114_amd import autotune
    a = autotune.cache_key(0, 30, [0, 700, 1500], 4)
    b = autotune.cache_key(0, 30, [0, 1024, 2000], 4)
    assert a == b == "p0|k30|T1024|c8"
    assert autotune.cache_key(0, 30, [0, 2049], 4) == "p0|k30|T4096|c4"
    assert autotune.cache_key(1, 30, [0, 700, 1500], 4) != a
    assert autotune.cache_key(0, 20, [0, 700, 1500], 4) != a
    assert {S for S, _ in autotune.SHAPES[_lib.RSV_F64]} == {4, 8}


def test_static_workspace_limit_checked_on_the_host():
    """rsv_hmc_init_static refuses a problem whose workspace exceeds the
    static array before any device call (no GPU needed)."""
    big = _pb([0, 1_200_000], max_steps=50)
    assert api.rsv_hmc_workspace_bytes(big) > _lib.RSV_STATIC_WORKSPACE_BYTES
    ctx = C.c_void_p()
    st = api.lib().rsv_hmc_init_static(C.byref(ctx), C.byref(big.struct()), None, None, None,
                                       None)
    assert st == _lib.RSV_ENOMEM and not ctx.value
    assert b"static workspace" in api.lib().rsv_last_error()
    small = _pb([0, 1000], max_steps=20)
    assert api.rsv_hmc_workspace_bytes(small) < _lib.RSV_STATIC_WORKSPACE_BYTES


def test_series_log_mass_falls_back_per_series():
    """Host logic of the learned-mass pipeline: a series with any non-finite
    network output takes the identity mass (ln m = 0) at every site; the
    other series keep theirs."""
    from paper_1603_08114_amd import learned_mass as LM
    off = np.array([0, 4, 9, 12])
    lm = np.arange(12, dtype=np.float32) / 10
    lm[6] = np.nan
    lm[11] = np.inf
    out, bad = LM.series_log_mass(lm, off)
    assert bad == [1, 2]
    assert np.array_equal(out[:4], lm[:4])
    assert np.all(out[4:] == 0.0)
    assert np.isnan(lm[6])  # the input is not modified
