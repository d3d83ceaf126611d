"""Pins of the oracle's random numbers.

Philox4x64-10 is checked word for word against numpy's independent
implementation of the same published generator; the uniform, normal and
Gamma transforms are checked against their distributions.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def _numpy_philox_block(ctr, key):
    """First block numpy produces from state counter `ctr`: numpy increments
    the 256-bit counter before encrypting, so this is Philox(ctr + 1, key)."""
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("ctr,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 7, 11, 13], [1, 2]),
    ([2**63 + 12345, 99, 3, 2], [0xDEADBEEFCAFEF00D, 0x0123456789ABCDEF]),
    ([2**64 - 1, 0, 0, 0], [3, 4]),                       # carry into word 1
    ([2**64 - 1, 2**64 - 1, 2**64 - 1, 17], [2**64 - 1, 2**64 - 1]),
])
def test_philox_matches_numpy(ctr, key):
    # numpy's next counter value, with carry, is what the oracle must be fed.
    c = list(ctr)
    for i in range(4):
        c[i] = (c[i] + 1) % 2**64
        if c[i] != 0:
            break
    ours = oracle.philox4x64_10(c, key)
    ref = _numpy_philox_block(ctr, key)
    assert np.array_equal(ours, ref), (ours, ref)


def test_philox_stream_many_counters():
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        c = [ctr[0] + 1] + ctr[1:]
        assert np.array_equal(oracle.philox4x64_10(c, key), _numpy_philox_block(ctr, key))


def test_uniforms_open_interval_and_ks():
    u = oracle.uniform_stream(seed=11, sweep=3, chain=5, tag=0, n=200_000)
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # the uniform is the top 52 bits of the word, centred: check exactly
    w = oracle.philox4x64_10([0, 3, 5, 0], [11, 0])
    expect = ((w >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0**-52
    assert np.array_equal(u[:4], expect)


def test_normals_ks_and_moments():
    z = oracle.normal_stream(seed=2, sweep=0, chain=9, tag=0, n=400_000)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    n = z.size
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / n)
    # Box-Muller pairs must be uncorrelated
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 4 / np.sqrt(n / 2)


def test_fp32_path_momenta_law():
    """The FP32-mixed path's layout (8 sites per Philox block, u0 from 40
    bits, u1 from 24): N(0, 1) by KS, mean, variance and kurtosis; the two
    normals of a pair uncorrelated, and so are neighbouring blocks; every
    radius within sqrt(-2 ln 2^-41), the smallest u0; and a stream apart
    from the FP64 layout's."""
    z = oracle.momenta_f32(seed=5, sweep=2, chain=3, T=400_000)
    n = z.size
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 4 * np.sqrt(2.0 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3.0) < 6 * np.sqrt(24.0 / n)
    assert abs(np.corrcoef(z[0::2], z[1::2])[0, 1]) < 4 / np.sqrt(n / 2)
    blocks = z.reshape(-1, 8)
    assert abs(np.corrcoef(blocks[:-1, 0], blocks[1:, 0])[0, 1]) < 4 / np.sqrt(blocks.shape[0])
    assert np.max(np.abs(z)) <= np.sqrt(2.0 * 41 * np.log(2.0))
    assert not np.allclose(z[:64], oracle.momenta(5, 2, 3, 64))


def test_streams_are_distinct():
    a = oracle.normal_stream(1, 0, 0, 0, 64)
    for (sw, ch, tag) in [(1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        b = oracle.normal_stream(1, sw, ch, tag, 64)
        assert not np.allclose(a, b)


@pytest.mark.parametrize("alpha", [1.0, 2.5, 26.0, 501.0])
def test_gamma_marsaglia_tsang_ks(alpha):
    n = 4000
    draws = np.empty(n)
    for i in range(n):
        v, exhausted = oracle.gamma(alpha, seed=5, sweep=i, chain=1)
        assert not exhausted
        draws[i] = v
    assert stats.kstest(draws, stats.gamma(alpha).cdf).pvalue > 1e-3
    assert abs(draws.mean() - alpha) < 4 * np.sqrt(alpha / n)
