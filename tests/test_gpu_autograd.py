"""The differentiable form through torch.autograd: FuelTimeCost's forward
against the oracle's fuel + time cost, its backward (the hand-written
adjoint) against the FP64 autograd transcription of the oracle on 32
particles and against central finite differences (h = 1e-4) of its own
forward, in an FP64 context."""
import numpy as np
import pytest

import synth
from oracle import grad as og
from oracle import rollout as ro
from tests.gpu_helpers import dev, host, separable_field

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case(lib):
    import torch
    from paper_1506_02869_amd import autograd as sag
    s = synth.shrink(synth.c4(precision="fp64"), M=4, H=40, S=4, grid=(8, 8, 4), L=32)
    fctx = sag.fuel_time_context(s)
    rng = np.random.default_rng(2)
    u = rng.uniform(0.15, 0.85, (32, s["N"], s["S"], 3))
    W = separable_field(s, 3)
    d = dict(W=dev(W), states=dev(s["states"]), k_active=dev(np.asarray(s["k_active"], np.int32)))
    return s, fctx, u, W, d, sag, torch


def test_forward_is_the_oracle_fuel_time_cost(case):
    s, fctx, u, W, d, sag, torch = case
    c = sag.fuel_time_cost(fctx, dev(u), d["W"], d["states"], d["k_active"])
    ref = ro.rollout(s, u, W)["ft_cost"].mean(axis=1)
    assert c.shape == (32, s["N"]) and c.dtype == torch.float64
    assert np.abs(host(c) - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-3)


def test_backward_matches_oracle_gradient(case):
    """Weighted sum of the outputs: the incoming gradient differs per
    (particle, aircraft), so the chain rule through the Function is checked
    too."""
    s, fctx, u, W, d, sag, torch = case
    ut = dev(u).requires_grad_(True)
    c = sag.fuel_time_cost(fctx, ut, d["W"], d["states"], d["k_active"])
    wts = np.random.default_rng(4).uniform(0.5, 2.0, (32, s["N"]))
    (c * dev(wts)).sum().backward()
    got = host(ut.grad)
    _, g = og.grad_fuel_time(s, u, W)            # d/du sum_i mean_m c_ft
    ref = g * wts[:, :, None, None]
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-9 * scale


def test_backward_matches_central_differences(case):
    """(F(u + h e) - F(u - h e)) / 2h of the GPU forward, h = 1e-4, on one
    random coordinate of each of the 32 particles; coordinates where the two
    one-sided differences disagree (a kink: landing, a clamp) are skipped
    and counted."""
    s, fctx, u, W, d, sag, torch = case
    ut = dev(u).requires_grad_(True)
    c = sag.fuel_time_cost(fctx, ut, d["W"], d["states"], d["k_active"])
    c.sum().backward()
    grad = host(ut.grad)
    rng = np.random.default_rng(7)
    h = 1e-4
    N, S = s["N"], s["S"]
    picks = [(l, int(rng.integers(N)), int(rng.integers(S)), int(rng.integers(3))) for l in range(32)]
    up = np.repeat(u[None], 3, axis=0).reshape(3 * 32, N, S, 3)
    for l, i, sg, k in picks:
        up[32 + l, i, sg, k] += h
        up[64 + l, i, sg, k] -= h
    F = host(sag.fuel_time_cost(fctx, dev(up), d["W"], d["states"], d["k_active"])).sum(axis=1)
    checked = skipped = 0
    scale = np.abs(grad).max()
    for l, i, sg, k in picks:
        f0, fp, fm = F[l], F[32 + l], F[64 + l]
        fwd, bwd = (fp - f0) / h, (f0 - fm) / h
        if abs(fwd - bwd) > 1e-3 * max(abs(fwd), abs(bwd), 1e-3 * scale):
            skipped += 1
            continue
        fd = (fp - fm) / (2 * h)
        assert abs(grad[l, i, sg, k] - fd) <= 1e-5 * scale + 1e-4 * abs(fd), (l, i, sg, k)
        checked += 1
    assert checked >= 24, (checked, skipped)
