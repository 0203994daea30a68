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


def test_mala_log_q_is_gaussian_in_logit_coordinates():
    rng = np.random.default_rng(2)
    a, b = rng.uniform(size=(5, 2, 3, 3)), rng.uniform(size=(5, 2, 3, 3))
    # logit and logistic are inverse maps of (0, 1) and R
    assert np.allclose(og.logistic(og.logit(a)), a, rtol=0, atol=1e-15)
    t = np.array([-800.0, -40.0, -1.0, 0.0, 2.5, 40.0, 800.0])
    assert np.allclose(og.logistic(t), 1.0 / (1.0 + np.exp(-np.clip(t, -700, 700))))
    # the u-gradient that makes the carried target flat: the drift vanishes
    g_flat = -(1.0 - 2.0 * a) / (a * (1.0 - a))
    assert np.allclose(og.mala_drift(a, g_flat, 0.3), 0.0, atol=1e-12)
    # a Gaussian density in theta, symmetric when both drifts vanish
    gb = -(1.0 - 2.0 * b) / (b * (1.0 - b))
    assert np.allclose(og.mala_log_q(a, b, gb, 0.1), og.mala_log_q(b, a, g_flat, 0.1))
    ga = rng.normal(size=a.shape)
    eps = 0.05
    ta, tb = np.log(a / (1 - a)), np.log(b / (1 - b))
    mean = ta + 0.5 * eps * eps * (ga * a * (1 - a) + 1 - 2 * a)
    ref = -np.sum(((tb - mean) ** 2).reshape(5, -1), axis=1) / (2 * eps * eps)
    assert np.allclose(og.mala_log_q(b, a, ga, eps), ref)
    # log |du/dtheta| = sum log u (1 - u)
    assert np.allclose(og.log_jacobian(a), np.log(a * (1 - a)).reshape(5, -1).sum(1))