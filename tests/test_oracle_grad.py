"""Pins of the reference gradient of the fuel + time cost: the PyTorch float64
transcription reproduces the NumPy oracle's value, and its autograd gradient
matches central finite differences (h = 1e-4) of the NumPy value on 32
random particles (components whose one-sided differences disagree, i.e. a
kink inside [-h, h], are skipped and counted)."""
import numpy as np
import pytest

import synth
from oracle import grad as og
from oracle import rollout as ro
from tests.gpu_helpers import separable_field


@pytest.fixture(scope="module")
def case():
    s = synth.shrink(synth.c4(precision="fp64"), M=3, H=40, S=4, grid=(8, 8, 4))
    rng = np.random.default_rng(0)
    u = rng.uniform(0.15, 0.85, (32, s["N"], s["S"], 3))
    W = separable_field(s, 1)
    return s, u, W


def test_torch_value_equals_numpy(case):
    s, u, W = case
    val, g = og.grad_fuel_time(s, u, W)
    r = ro.rollout(s, u, W)
    assert np.abs(val - r["ft_cost"].mean(axis=1)).max() < 1e-14
    assert g.shape == u.shape and np.isfinite(g).all()


def test_gradient_matches_central_differences(case):
    s, u, W = case
    _, g = og.grad_fuel_time(s, u, W)
    rng = np.random.default_rng(1)
    h = 1e-4
    checked = skipped = 0
    for l in range(32):
        i = int(rng.integers(s["N"]))
        sg = int(rng.integers(s["S"]))
        c = int(rng.integers(3))
        f = lambda uu: ro.rollout(s, uu[l:l + 1], W)["ft_cost"].mean(axis=1)[0].sum()
        up, um = u.copy(), u.copy()
        up[l, i, sg, c] += h
        um[l, i, sg, c] -= h
        f0, fp, fm = f(u), f(up), f(um)
        d_plus, d_minus = (fp - f0) / h, (f0 - fm) / h
        fd = (fp - fm) / (2 * h)
        if abs(d_plus - d_minus) > 1e-3 * max(abs(fd), 1e-3):
            skipped += 1          # a kink (max(T, 0), min(t, 1), landing) inside
            continue
        assert abs(fd - g[l, i, sg, c]) <= 1e-5 * max(abs(fd), 1e-4), (l, i, sg, c)
        checked += 1
    assert checked >= 24 and skipped <= 8


def test_mala_log_q_is_gaussian():
    rng = np.random.default_rng(2)
    a, b = rng.uniform(size=(5, 2, 3, 3)), rng.uniform(size=(5, 2, 3, 3))
    g = np.zeros_like(a)
    # symmetric without drift
    assert np.allclose(og.mala_log_q(a, b, g, 0.1), og.mala_log_q(b, a, g, 0.1))
    ga = rng.normal(size=a.shape)
    eps = 0.05
    mean = a + 0.5 * eps * eps * ga
    ref = -np.sum(((b - mean) ** 2).reshape(5, -1), axis=1) / (2 * eps * eps)
    assert np.allclose(og.mala_log_q(b, a, ga, eps), ref)
