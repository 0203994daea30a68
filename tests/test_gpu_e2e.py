"""End-to-end GPU parity: whole MPC updates through smc_mpc_step and
smc_eval_cost against the oracle, full-size sampled rollouts, determinism and
the degenerate cases."""
import numpy as np
import pytest

import synth
from oracle import rollout as oro
from oracle import smc as osmc
from tests.gpu_helpers import dev, empty, host, rel_err, separable_field, zeros

pytestmark = pytest.mark.gpu


def _norm(scen, ctrl):
    lo, hi = scen["ctrl_lo"], scen["ctrl_hi"]
    return (ctrl - lo) / (hi - lo)


@pytest.mark.parametrize("move", [0, 1])
def test_c1_fp64_step_matches_oracle(lib, move):
    """C1 in FP64: returned controls within 1e-4 (normalised units) and
    expected cost within 1e-5 relative of the oracle's whole SMC run."""
    s = synth.c1(move="jitter" if move == 0 else "rwmh")
    if move == 1:
        s = synth.shrink(s, K=10)
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    assert status == (1 if ref["infeasible"] else 0)
    assert info["best_particle"] == ref["best"]
    assert np.abs(_norm(s, ctrl) - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)
    assert np.all(rel_err(cost[1:], ref["cost_per"]) < 1e-5)


def test_step_is_deterministic_and_reports_work(lib):
    s = synth.shrink(synth.c2(), L=512, M=8, K=4)
    ctx = lib.smc_mpc_init(s)
    a = lib.smc_mpc_step(ctx)
    b = lib.smc_mpc_step(ctx)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[3]["aircraft_steps"] > 0 and a[3]["ms_total"] > 0
    c = lib.smc_mpc_step(ctx, mpc_step=1)
    assert not np.array_equal(a[0], c[0])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eval_cost_matches_oracle(lib, prec):
    s = synth.shrink(synth.c2(precision=prec), M=6, grid=(8, 8, 4))
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(3)
    P = 23
    parts = rng.uniform(0, 1, (P, s["N"], s["S"], 3))
    if prec == "fp32":
        parts = parts.astype(np.float32).astype(np.float64)
    cost, feas = lib.smc_eval_cost(ctx, parts, 7)
    rc, rf = osmc.eval_cost(s, parts, 7)
    ok = feas == rf
    assert ok.mean() > 0.9
    assert np.all(rel_err(cost, rc)[ok] < (1e-6 if prec == "fp64" else 2e-5))


def _check_sampled_worlds(s, u, W, cost_at, feas_at, picks):
    """Compare the (particle, sample) worlds in picks with the oracle one by
    one: feasibility exactly, per-aircraft cost within 2e-5 relative (FP32),
    skipping worlds with a discrete decision within 1e-4 of its threshold.
    Returns the number of worlds compared."""
    bad = compared = 0
    for (p, m) in picks:
        r = oro.rollout(s, u[p:p + 1].astype(np.float64), W[m:m + 1].astype(np.float64),
                        with_margins=True)
        if (r["margin"] < 1e-4).any():
            continue
        compared += 1
        assert np.array_equal(feas_at(p, m), r["feas"][0, 0]), (p, m)
        e = rel_err(cost_at(p, m), r["cost"][0, 0])
        bad += int((e > 2e-5).sum())
    assert bad == 0
    return compared


@pytest.mark.parametrize("layout", [0, 1])
def test_full_size_c2_rollout_sampled(lib, layout):
    """C2 at full size (8192 particles x 64 wind samples x 10 aircraft x 120
    steps; layout 0 is the launch the benchmark times); 48 random worlds are
    checked against the oracle one by one."""
    import torch
    s = synth.c2()
    ctx = lib.smc_mpc_init(s)
    lib.smc_set_rollout_layout(ctx, layout)
    P, M, N, S = s["L"], s["M"], s["N"], s["S"]
    rng = np.random.default_rng(11)
    u = rng.uniform(0, 1, (P, N, S, 3)).astype(np.float32)
    W = separable_field(s, 5).astype(np.float32)
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    lib.smc_k_rollout(ctx, dev(u), P, dev(W), dev(s["states"]), dev(s["k_active"]), s["H"],
                      cost, feas)
    gc, gf = host(cost), host(feas).astype(bool)
    picks = [(int(rng.integers(P)), int(rng.integers(M))) for _ in range(48)]
    picks += [(0, 0), (P - 1, M - 1)]
    n = _check_sampled_worlds(s, u, W, lambda p, m: gc[m, p], lambda p, m: gf[m, p], picks)
    assert n >= 40


def test_full_size_c4_rollout_and_adjoint_sampled(lib):
    """C4 at full size (16384 particles x 64 wind samples x 20 aircraft x 150
    steps: the 20-aircraft world-per-lane rollout and the adjoint, the
    launches the benchmark times).  24 random worlds against the oracle's
    rollout; the summed fuel + time gradient of 4 random particles (all
    aircraft, all 64 samples) against the FP64 autograd reference, excluding
    aircraft with a landing decision within 1e-4 of its threshold."""
    import torch
    from oracle import grad as og
    s = synth.c4()
    ctx = lib.smc_mpc_init(s)
    P, M, N, S = s["L"], s["M"], s["N"], s["S"]
    rng = np.random.default_rng(12)
    u = rng.uniform(0, 1, (P, N, S, 3)).astype(np.float32)
    W = separable_field(s, 6).astype(np.float32)
    du, dW = dev(u), dev(W)
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    lib.smc_k_rollout(ctx, du, P, dW, dev(s["states"]), dev(s["k_active"]), s["H"], cost, feas)
    g = empty((P, N, S, 3), torch.float64)
    lib.smc_k_rollout_grad(ctx, du, P, dW, dev(s["states"]), dev(s["k_active"]), s["H"], g)
    gc, gf, gg = host(cost), host(feas).astype(bool), host(g)
    picks = [(int(rng.integers(P)), int(rng.integers(M))) for _ in range(22)]
    picks += [(0, 0), (P - 1, M - 1)]
    n = _check_sampled_worlds(s, u, W, lambda p, m: gc[m, p], lambda p, m: gf[m, p], picks)
    assert n >= 16
    W64 = W.astype(np.float64)
    checked = 0
    for p in [int(x) for x in rng.integers(P, size=4)]:
        u64 = u[p:p + 1].astype(np.float64)
        r = oro.rollout(s, u64, W64, with_margins=True)
        keep = (r["margin"][0] >= 1e-4).all(axis=0)          # per aircraft, over samples
        _, ref = og.grad_fuel_time(s, u64, W64)
        ref = ref[0] * M                                     # sum over the samples
        got = gg[p]
        scale = np.abs(ref[keep]).max()
        err = np.abs(got[keep] - ref[keep])
        assert err.max() <= 2e-3 * scale, (p, err.max() / scale)
        assert np.median(err / np.maximum(np.abs(ref[keep]), 1e-3 * scale)) < 1e-4
        checked += int(keep.sum())
    assert checked >= 60


def test_full_size_c5_rollout_sampled(lib):
    """C5 at full size (65536 particles x 128 wind samples x 40 aircraft x
    180 steps, 780 pairs, noise term over a 256 x 256 population grid: the
    aircraft-per-lane rollout the benchmark times); 24 random worlds against
    the oracle one by one (sampled on the device, only they are copied)."""
    import torch
    s = synth.c5()
    ctx = lib.smc_mpc_init(s)
    P, M, N, S = s["L"], s["M"], s["N"], s["S"]
    rng = np.random.default_rng(13)
    u = rng.uniform(0, 1, (P, N, S, 3)).astype(np.float32)
    W = separable_field(s, 7).astype(np.float32)
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    lib.smc_k_rollout(ctx, dev(u), P, dev(W), dev(s["states"]), dev(s["k_active"]), s["H"],
                      cost, feas)
    picks = [(int(rng.integers(P)), int(rng.integers(M))) for _ in range(22)]
    picks += [(0, 0), (P - 1, M - 1)]
    # the rollout ran on the context's own stream: wait for it before torch
    # gathers the sampled worlds on its stream
    torch.cuda.synchronize()
    pi = torch.as_tensor([p for p, _ in picks], device=cost.device)
    mi = torch.as_tensor([m for _, m in picks], device=cost.device)
    sc, sf = host(cost[mi, pi]), host(feas[mi, pi]).astype(bool)
    at = {pm: k for k, pm in enumerate(picks)}
    n = _check_sampled_worlds(s, u, W, lambda p, m: sc[at[(p, m)]],
                              lambda p, m: sf[at[(p, m)]], picks)
    assert n >= 12


def test_all_infeasible_returns_warning(lib):
    """Two aircraft at the same point and altitude: every particle violates
    separation at the first step; the update still returns a particle."""
    s = synth.shrink(synth.c1(), L=64, K=3)
    st = s["states"].copy()
    st[1] = st[0]
    s = dict(s, states=st, kind=np.array([1, 1], np.int8))
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    assert status == lib.SMC_INFEASIBLE
    assert info["feasible_frac"] == 0.0
    ref = osmc.smc_mpc_step(s)
    assert ref["infeasible"]
    assert info["best_particle"] == ref["best"]


def test_inactive_and_late_aircraft(lib):
    s = synth.shrink(synth.c2(), L=128, M=4, K=3, grid=(8, 8, 4))
    ka = s["k_active"].copy()
    ka[0] = -1        # not in the problem
    ka[1] = 200       # beyond the horizon
    ka[2] = 119       # enters at the last step
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx, k_active=ka)
    assert cost[1] == 0.0 and cost[2] == 0.0
    assert np.isfinite(cost).all()


def test_short_horizon_and_errors(lib):
    s = synth.c1()
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx, horizon=6)
    assert np.isfinite(cost).all()
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_step(ctx, horizon=61)
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_step(ctx, horizon=5)   # fewer steps than segments
