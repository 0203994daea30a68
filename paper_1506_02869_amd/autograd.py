"""The differentiable form: a torch.autograd.Function whose forward is the
GPU rollout's fuel + time-to-go cost and whose backward is the hand-written
adjoint of the same rollout (smc_k_rollout_grad).

Build addition (the paper's optimiser is derivative-free; Sec. "Particle
Costing" defines the fuel element and the cost weighting).  The forward runs
the rollout kernel under a companion context whose cost keeps only the
differentiable elements: the heading, glide, bearing, altitude, speed and
noise weights are zero and the fuel weights are rescaled so that the fuel
element's coefficient (1 - alpha_time - alpha_noise) w_fuel is unchanged.
Its per-world cost is then exactly the fuel + time part the adjoint
differentiates, and the forward returns its mean over the wind samples,
c_ft[p, i] = (1/M) sum_m cost_ft[m, p, i] (Kahan FP64 sum, smc_k_reduce).

Argument marshalling and the chain rule only: both passes run in the HIP
kernels behind the C ABI.
"""
from __future__ import annotations

import numpy as np
import torch

from . import smc_k_reduce, smc_k_rollout, smc_k_rollout_grad, smc_mpc_init

_FUEL_ARR, _FUEL_DEP, _TIME, _NOISE = 2, 4, 7, 8


def fuel_time_scenario(scen: dict) -> dict:
    """The scenario whose cost is the fuel + time-to-go part of `scen`'s."""
    s = dict(scen)
    w = np.array(scen["cost_w"], dtype=np.float64).copy()
    keep = (1.0 - w[_TIME] - w[_NOISE]) / (1.0 - w[_TIME])
    w[_FUEL_ARR] *= keep
    w[_FUEL_DEP] *= keep
    for k in range(len(w)):
        if k not in (_FUEL_ARR, _FUEL_DEP, _TIME):
            w[k] = 0.0
    s["cost_w"] = w
    return s


def fuel_time_context(scen: dict):
    """Companion context of a scenario for FuelTimeCost (same sizes,
    precision, grid and aircraft; fuel + time cost only)."""
    return smc_mpc_init(fuel_time_scenario(scen))


class FuelTimeCost(torch.autograd.Function):
    """c_ft = FuelTimeCost.apply(u, W, states, k_active, horizon, fctx).

    u: normalised controls [P, N, S, 3] in the context's precision (device);
    W: wind fields [M, G, 2]; states [N, 6] float64; k_active [N] int32;
    fctx: a fuel_time_context.  Returns c_ft [P, N] float64, the mean over
    the M samples of each aircraft's fuel + time-to-go cost.  The gradient
    with respect to u is the adjoint's sum over the samples divided by M,
    scaled by the incoming gradient of each (particle, aircraft) (aircraft
    i's cost depends only on its own controls).  Landing carries no
    derivative and clamps take the active branch, as in the adjoint."""

    @staticmethod
    def forward(fc, u, W, states, k_active, horizon, fctx):
        P = int(u.shape[0])
        dev = u.device
        uc = u.detach().contiguous()
        cost = torch.empty((fctx.M, P, fctx.N), dtype=torch.float64, device=dev)
        feas = torch.empty((fctx.M, P, fctx.N), dtype=torch.uint8, device=dev)
        smc_k_rollout(fctx, uc, P, W, states, k_active, int(horizon), cost, feas)
        chat = torch.empty((P, fctx.N), dtype=torch.float64, device=dev)
        fpn = torch.empty((P, fctx.N), dtype=torch.uint8, device=dev)
        logw = torch.empty((P, fctx.N), dtype=torch.float64, device=dev)
        smc_k_reduce(fctx, P, cost, feas, 0.0, chat, fpn, logw)
        fc.save_for_backward(uc, W, states, k_active)
        fc.fctx, fc.horizon = fctx, int(horizon)
        return chat

    @staticmethod
    def backward(fc, grad_out):
        uc, W, states, k_active = fc.saved_tensors
        fctx = fc.fctx
        P = int(uc.shape[0])
        g = torch.empty((P, fctx.N, fctx.S, 3), dtype=torch.float64, device=uc.device)
        smc_k_rollout_grad(fctx, uc, P, W, states, k_active, fc.horizon, g)
        gu = g * (grad_out.to(torch.float64) / fctx.M)[:, :, None, None]
        return gu.to(uc.dtype), None, None, None, None, None


def fuel_time_cost(fctx, u, W, states, k_active, horizon=None):
    """Differentiable fuel + time cost c_ft [P, N] (see FuelTimeCost)."""
    return FuelTimeCost.apply(u, W, states, k_active,
                              fctx.H if horizon is None else horizon, fctx)
