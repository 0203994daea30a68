"""GPU parity of the gradient-informed form: the hand-written adjoint against
the FP64 autograd reference (itself pinned by finite differences), the
Langevin proposal / acceptance kernels, and whole MALA updates."""
import numpy as np
import pytest

import synth
from oracle import grad as og
from oracle import smc as osmc
from tests.gpu_helpers import dev, empty, host, separable_field

pytestmark = pytest.mark.gpu


def _grad_case(lib, prec, M=3, P=7, H=40, S=4, seed=0, **scen_kw):
    import torch
    s = synth.shrink(synth.c4(precision=prec, **scen_kw), M=M, H=H, S=S, grid=(8, 8, 4),
                     L=max(P, 2))
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.15, 0.85, (P, s["N"], s["S"], 3))
    W = separable_field(s, seed + 1)
    if prec == "fp32":
        u = u.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    g = empty((P, s["N"], s["S"], 3), torch.float64)
    lib.smc_k_rollout_grad(ctx, dev(u, ctx.real_dtype), P, dev(W, ctx.real_dtype),
                           dev(s["states"]), dev(s["k_active"]), s["H"], g)
    _, ref = og.grad_fuel_time(s, u, W)
    return host(g), ref * M


def _grad_case_events(lib, prec, M, H, S=6, P=5):
    """An arrival placed 14 km out on the runway axis, flying in at 120 m/s
    and descending, lands after 12 ... 14 steps depending on the sample; one
    aircraft joins at step 37, one never does, one joins 3 steps before the
    end."""
    import torch
    s = synth.shrink(synth.c4(precision=prec), M=M, H=H, S=S, grid=(8, 8, 4), L=P)
    s["states"] = s["states"].copy()
    s["k_active"] = s["k_active"].copy()
    assert s["kind"][0] == 0 and s["kind"][13] == 1
    s["states"][0, :5] = [14000.0, 0.0, 700.0, 120.0, np.pi]
    s["k_active"][1] = 37
    s["k_active"][2] = -1
    s["k_active"][13] = H - 3
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(5)
    u = rng.uniform(0.15, 0.85, (P, s["N"], s["S"], 3))
    u[:, 0, :, :] = [0.5, 0.05, 0.4]     # no turn, 117 m/s commanded, -3 m/s climb
    W = separable_field(s, 6)
    if prec == "fp32":
        u = u.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    g = empty((P, s["N"], s["S"], 3), torch.float64)
    lib.smc_k_rollout_grad(ctx, dev(u, ctx.real_dtype), P, dev(W, ctx.real_dtype),
                           dev(s["states"]), dev(s["k_active"]), s["H"], g)
    _, ref = og.grad_fuel_time(s, u, W)
    return host(g), ref * M


# M = 40 and 64 with H <= 160: one wave per (particle, aircraft) (the last
# 8-step block ragged at H = 157); M = 24: two per wave; M = 80: a two-wave
# workgroup per (particle, aircraft); H = 161: the per-lane form
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,H", [(40, 157), (64, 160), (24, 157), (80, 157), (40, 161)])
def test_adjoint_landing_late_and_inactive_aircraft(lib, prec, M, H):
    got, ref = _grad_case_events(lib, prec, M, H)
    assert np.all(got[:, 2] == 0.0) and np.all(ref[:, 2] == 0.0)   # never active
    # FP32: a sample that meets a discrete decision of the derivative (the
    # grid clamp, the thrust floor, the time element's cap) on the other side
    # than the FP64 oracle moves its group's sum by up to about 1/M of the
    # group's scale (1.3 % for the late joiner at M = 64, the same with the
    # per-lane form; 0.5 % of the largest gradient at M = 24); the median
    # error stays at rounding level
    tol = 1e-9 if prec == "fp64" else max(2e-2, 1.0 / M)
    for i in (0, 1, 13):   # the landing, late and last-moment aircraft, each on its own scale
        sc = np.abs(ref[:, i]).max()
        assert sc > 0.0
        assert np.abs(got[:, i] - ref[:, i]).max() <= tol * sc, i
    sc = np.abs(ref).max()
    err = np.abs(got - ref)
    assert err.max() <= tol * sc
    if prec == "fp32":
        assert np.median(err / np.maximum(np.abs(ref), 1e-3 * sc)) < 1e-4


# two (particle, aircraft) per wave (17 ... 32 samples), an odd number of
# them (5 particles x 5 aircraft): the last wave's upper half is empty
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_adjoint_two_groups_per_wave_odd_count(lib, prec):
    got, ref = _grad_case(lib, prec, M=24, P=5, H=150, S=6, n_arr=3, n_dep=2)
    assert got.shape[1] == 5
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    # FP32: up to one sample in M on the other side of a discrete decision
    # of the derivative than the FP64 oracle (see the test above)
    assert err.max() <= (1e-9 if prec == "fp64" else 1.0 / 24) * scale
    if prec == "fp32":
        assert np.median(err / np.maximum(np.abs(ref), 1e-3 * scale)) < 1e-4


@pytest.mark.parametrize("M,H", [(3, 40), (16, 40), (80, 40), (64, 150), (32, 150)])
def test_adjoint_fp64_matches_reference(lib, M, H):
    got, ref = _grad_case(lib, "fp64", M=M, P=5 if M == 80 else 7, H=H,
                          S=6 if H > 100 else 4)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-9 * scale


# (M, H, S): segment checkpoints in registers up to 6 segments (H <= 150),
# in scratch memory beyond; one wave per (particle, aircraft) at M = 64
@pytest.mark.parametrize("M,H,S", [(8, 40, 4), (64, 150, 6), (5, 180, 6), (100, 150, 6)])
def test_adjoint_fp32_matches_reference(lib, M, H, S):
    got, ref = _grad_case(lib, "fp32", M=M, H=H, S=S)
    scale = np.abs(ref).max()
    err = np.abs(got - ref)
    assert err.max() <= 2e-3 * scale
    assert np.median(err / np.maximum(np.abs(ref), 1e-3 * scale)) < 1e-4


def test_mala_kernels_match_oracle(lib):
    import torch
    s = synth.shrink(synth.c1(move="mala"), L=64, K=4)
    ctx = lib.smc_mpc_init(s)
    P, N, S = 64, s["N"], s["S"]
    rng = np.random.default_rng(4)
    u = rng.uniform(0.05, 0.95, (P, N, S, 3))
    G = rng.normal(size=(P, N, S, 3)) * 3.0
    beta, J, step = 9.0, 2, 1
    up = empty((P, N, S, 3), torch.float64)
    lib.smc_k_mala_propose(ctx, P, dev(u), dev(G), beta, up, step, J)
    g = -beta * G / s["M"]
    ref_up = osmc.mala_propose(s, u, g, J, mpc_step=step)
    up_h = host(up)
    assert np.abs(up_h - ref_up).max() < 1e-14
    Gp = rng.normal(size=(P, N, S, 3)) * 3.0
    chat = rng.uniform(0, 1, (P, N))
    chat2 = chat + rng.normal(0, 0.01, (P, N))
    f1 = np.ones((P, N), bool)
    f2 = rng.uniform(size=(P, N)) > 0.05
    l1 = osmc.log_weights(chat, f1, beta)
    l2 = osmc.log_weights(chat2, f2, beta)
    gp = -beta * Gp / s["M"]
    inside, lq = osmc.mala_log_ratio(s, u, ref_up, g, gp)
    acc_ref = osmc.mh_accept(s, J, l1, np.where(inside[:, None], l2, -np.inf), mpc_step=step,
                             log_q_ratio=lq)
    acc = empty((P,), torch.int32)
    d_u = dev(u)
    lib.smc_k_mala_accept(ctx, P, d_u, up, dev(G), dev(Gp), beta, dev(chat), dev(chat2),
                          dev(f1.astype(np.uint8)), dev(f2.astype(np.uint8)), dev(l1), dev(l2),
                          step, J, acc)
    assert np.array_equal(host(acc).astype(bool), acc_ref)
    assert 0 < acc_ref.sum() < P


def test_mala_step_matches_oracle(lib):
    """A whole FP64 MPC update with Langevin moves on a C1-shaped scenario."""
    s = synth.shrink(synth.c1(move="mala"), L=64, K=5, H=30, S=3, M=4)
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    assert info["best_particle"] == ref["best"]
    u = (ctrl - s["ctrl_lo"]) / (s["ctrl_hi"] - s["ctrl_lo"])
    assert np.abs(u - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)
    assert 0.0 < info["accept_rate"] <= 1.0
