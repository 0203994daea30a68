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
    bad = 0
    for (p, m) in picks:
        r = oro.rollout(s, u[p:p + 1].astype(np.float64), W[m:m + 1].astype(np.float64),
                        with_margins=True)
        if (r["margin"] < 1e-4).any():
            continue
        assert np.array_equal(gf[m, p], r["feas"][0, 0])
        e = rel_err(gc[m, p], r["cost"][0, 0])
        bad += int((e > 2e-5).sum())
    assert bad == 0


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
