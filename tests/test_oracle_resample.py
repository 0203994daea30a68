"""Pins of the oracle's per-aircraft systematic resampling (Sec. "Particle
Resampling and Perturbation")."""
import math

import numpy as np
import pytest

from oracle import smc


def _mult(anc, L):
    return np.bincount(anc, minlength=L)


@pytest.mark.parametrize("L", [1, 2, 5, 64, 257, 1000])
def test_counts_and_bounds(L):
    rng = np.random.default_rng(L)
    for _ in range(5):
        logw = rng.normal(0, 3, L)
        logw[rng.uniform(size=L) < 0.2] = -np.inf
        if not np.isfinite(logw).any():
            logw[0] = 0.0
        U = int(rng.integers(0, 2**32))
        anc = smc.resample_row(logw, U)
        n = _mult(anc, L)
        assert n.sum() == L
        assert np.all(np.diff(anc) >= 0)                 # non-decreasing
        assert np.all(n[~np.isfinite(logw)] == 0)        # zero weight never chosen
        q = np.array(smc.quantised_weights(logw), dtype=object)
        Q = int(sum(q))
        for l in range(L):
            lo = (L * int(q[l])) // Q
            assert n[l] in (lo, lo + 1)


def test_unbiased_over_offsets():
    """E_U[N_l] = L q_l / Q, averaging over a regular grid of offsets."""
    L = 7
    logw = np.log(np.array([0.05, 0.3, 0.0001, 0.2, 0.15, 0.2, 0.0999]))
    q = smc.quantised_weights(logw)
    Q = sum(q)
    acc = np.zeros(L)
    n_u = 4096
    for t in range(n_u):
        U = (t * (2**32 // n_u)) + 12345
        acc += _mult(smc.resample_row(logw, U), L)
    assert np.allclose(acc / n_u, L * np.array(q) / Q, atol=L / n_u * 2)


def test_special_cases():
    L = 50
    for U in (0, 1, 2**31, 2**32 - 1):
        assert np.array_equal(smc.resample_row(np.zeros(L), U), np.arange(L))
        one = np.full(L, -np.inf)
        one[17] = -3.0
        assert np.all(smc.resample_row(one, U) == 17)
        assert np.array_equal(smc.resample_row(np.full(L, -np.inf), U), np.arange(L))


def test_matches_textbook_float_systematic_resampling():
    """Away from ties at thresholds, the exact integer form agrees with the
    usual floating-point systematic resampling (search of (k + u)/L in the
    normalised cumulative weights)."""
    rng = np.random.default_rng(3)
    for L in (10, 100, 4096):
        w = rng.gamma(0.5, size=L)
        U = int(rng.integers(0, 2**32))
        anc = smc.resample_row(np.log(w), U)
        cw = np.cumsum(w / w.sum())
        pts = (np.arange(L) + U / 2**32) / L
        ref = np.searchsorted(cw, pts, side="right")
        gap = np.min(np.abs(cw[:, None] - pts[None, :]))
        assert gap > 1e-12
        assert np.array_equal(anc, np.minimum(ref, L - 1))


def test_quantisation_exactness():
    for L in (2, 1000, 65536):
        kq = smc.quant_bits(L)
        assert L * 2**kq <= 2**52
        q = smc.quantised_weights(np.zeros(L))
        assert sum(q) == L * 2**kq
        # the fp64 running sum is exact: equals the integer running sum
        rng = np.random.default_rng(L)
        qq = smc.quantised_weights(rng.normal(0, 2, L))
        f = np.cumsum(np.array(qq, dtype=np.float64))
        assert all(int(a) == b for a, b in zip(f, np.cumsum(np.array(qq, dtype=object))))
