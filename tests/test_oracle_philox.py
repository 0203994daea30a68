"""Pins of the oracle's Philox4x32-10 generator and its transforms.

No published known-answer vectors are available in this environment, so the
generator is pinned by properties a wrong multiplier, a swapped output word,
a missing key bump or a 64-bit overflow would break: bijectivity of the
counter map, bit balance, avalanche, uniform and normal goodness of fit.
"""
import math

import numpy as np
from scipy import stats

from oracle import philox


def _words(n, J=0, purpose=philox.WIND, seed=0, step=0):
    return philox.words(seed, step, J, purpose, np.arange(n, dtype=np.int64))


def _scalar_round_trip(c, k):
    """Scalar Python-int transcription, to check the vectorised uint64 path
    does not overflow or truncate (not a pin of the definition itself)."""
    c = list(c)
    k0, k1 = k
    for r in range(10):
        if r:
            k0 = (k0 + 0x9E3779B9) & 0xFFFFFFFF
            k1 = (k1 + 0xBB67AE85) & 0xFFFFFFFF
        p0 = 0xD2511F53 * c[0]
        p1 = 0xCD9E8D57 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 & 0xFFFFFFFF, (p0 >> 32) ^ c[3] ^ k1,
             p0 & 0xFFFFFFFF]
    return c


def test_vectorised_matches_scalar_ints():
    rng = np.random.default_rng(1)
    C = rng.integers(0, 2**32, size=(64, 4), dtype=np.uint64)
    K = rng.integers(0, 2**32, size=2, dtype=np.uint64)
    out = philox.philox4x32_10(C[:, 0], C[:, 1], C[:, 2], C[:, 3], int(K[0]), int(K[1]))
    for n in range(64):
        ref = _scalar_round_trip([int(v) for v in C[n]], (int(K[0]), int(K[1])))
        assert [int(o[n]) for o in out] == ref


def test_counter_map_is_injective_on_a_sample():
    w = _words(200_000)
    packed = set(zip(*(x.tolist() for x in w)))
    assert len(packed) == 200_000


def test_bit_balance_and_avalanche():
    w = np.stack(_words(100_000)).astype(np.uint64)
    bits = ((w[..., None] >> np.arange(32, dtype=np.uint64)) & np.uint64(1)).astype(np.float64)
    frac = bits.mean(axis=1)                          # per word, per bit
    # binomial 3-sigma band for n = 1e5
    assert np.all(np.abs(frac - 0.5) < 4 * math.sqrt(0.25 / 100_000))
    # flipping one counter bit flips about half of the 128 output bits
    base = np.arange(20_000, dtype=np.int64) * 2
    a = np.stack(philox.words(0, 0, 0, 2, base)).astype(np.uint64)
    b = np.stack(philox.words(0, 0, 0, 2, base + 1)).astype(np.uint64)
    x = a ^ b
    flips = sum(((x >> np.uint64(s)) & np.uint64(1)).sum(axis=0) for s in range(32))
    assert abs(flips.mean() - 64.0) < 0.5
    # distinct streams (iteration J, purpose, MPC step, seed) decorrelated
    for other in (dict(J=1), dict(purpose=philox.MOVE), dict(step=1), dict(seed=1)):
        y = np.stack(_words(20_000, **other)).astype(np.float64)
        z = np.stack(_words(20_000)).astype(np.float64)
        r = np.corrcoef(y[0], z[0])[0, 1]
        assert abs(r) < 0.03
        assert not np.any(y[0] == z[0]) or (y[0] == z[0]).mean() < 1e-3


def test_uniforms_open_interval_and_goodness_of_fit():
    u = philox.uniforms(7, 3, 5, philox.INIT, np.arange(200_000))
    assert u.min() > 0.0 and u.max() < 1.0
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    assert abs(u.mean() - 0.5) < 4 * math.sqrt(1 / 12 / 200_000)
    # extreme words map to the documented end points
    lo = philox.uniform_from(np.uint32(0), np.uint32(0))
    hi = philox.uniform_from(np.uint32(0xFFFFFFFF), np.uint32(0xFFFFFFFF))
    assert lo == 0.5 * 2.0 ** -52
    assert hi == 1.0 - 0.5 * 2.0 ** -52


def test_box_muller_normals():
    z0, z1 = philox.normals_pair(0, 0, 0, philox.WIND, np.arange(200_000))
    for z in (z0, z1):
        assert stats.kstest(z, "norm").pvalue > 1e-3
        assert abs(z.mean()) < 0.015 and abs(z.var() - 1) < 0.015
    assert abs(np.corrcoef(z0, z1)[0, 1]) < 0.015
