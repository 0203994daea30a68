"""GPU parity of the paper's time-correlated wind model (Sec. "Wind Model":
exponential covariance eq. cov, linear Gaussian time recursion): the fields
of an iteration, the rollout that reads one field per step, and whole MPC
updates, each against the oracle."""
import numpy as np
import pytest

import synth
from oracle import rollout as oro
from oracle import smc as osmc
from oracle import wind as owind
from tests.gpu_helpers import dev, empty, host, rel_err, zeros

pytestmark = pytest.mark.gpu


def _ar1(base, prec="fp64", **kw):
    return synth.shrink(base(precision=prec, wind_model="ar1"), **kw)


def _field_bound(Q, V, a):
    """Upper bound of |u(k)| by the recursion on |v| (test tolerance only),
    pushed through |Qhat|: [H, G, M, 2]."""
    b = np.sqrt(1.0 - a * a)
    U = np.empty_like(V)
    for k in range(V.shape[0]):
        U[k] = np.abs(V[k]) if k == 0 else a * U[k - 1] + b * np.abs(V[k])
    H, G, M, _ = V.shape
    return np.stack([(np.abs(Q) @ U[k].reshape(G, 2 * M)).reshape(G, M, 2) for k in range(H)])


@pytest.mark.parametrize("prec,grid,M,H", [("fp64", (6, 5, 3), 4, 12), ("fp32", (6, 5, 3), 4, 12),
                                           ("fp64", (16, 16, 4), 16, 60),
                                           ("fp32", (16, 16, 4), 16, 60),
                                           ("fp32", (32, 32, 8), 4, 16)])
def test_fields_match_oracle(lib, prec, grid, M, H):
    """Every step's field of one iteration (the C1 grid at its own sample
    count and horizon, and the full C2 grid) against the oracle's recursion
    on the fields: within the rounding of the G-term products, plus the
    sensitivity of the Cholesky factors to the order of their operations
    (the library factors on the host in its own order), to first order
    u kappa for a factor of a matrix with condition number kappa."""
    s = _ar1(synth.c1, prec, grid=grid, M=M, H=H, S=min(6, H))
    s["wind_mean"] = np.array([2.0, -1.0])
    ctx = lib.smc_mpc_init(s)
    G = ctx.G
    W = empty((H, M, G, 2), ctx.real_dtype)
    lib.smc_k_wind_fields(ctx, s["mpc_step"], 3, s["wind_mean"], W)
    got = host(W).astype(np.float64)
    Q = owind.factor(s)
    a = owind.ar1_coefficient(s["dt"], s["wind_tcorr"])
    ref = owind.sample_field(s, 3, Lfac=Q)
    V = owind.ar1_normals(s["seed"], s["mpc_step"], 3, G, M, H)
    bound = _field_bound(Q, V, a).transpose(0, 2, 1, 3)          # [H, M, G, 2]
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    ax, ay, az = owind.grid_axes(s["box"], s["grid"])
    kap = (np.linalg.cond(owind.exp_gram_h(ax, ay, s["wind_beta"]) + s["wind_nugget"] * np.eye(len(ax) * len(ay)))
           + np.linalg.cond(owind.exp_gram_z(az, s["wind_gamma"]) + s["wind_nugget"] * np.eye(len(az))))
    tol = (2 * u * (4 + np.sqrt(G) + H) + 4 * 2.0 ** -53 * kap) * bound + u * np.abs(ref)
    err = np.abs(got - ref)
    assert np.all(err <= tol), (err.max(), (err / tol).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["c1", "c2", "c2-short"])
def test_rollout_reads_one_field_per_step(lib, prec, which):
    """The oracle's per-step fields in, cost and feasibility out, against the
    oracle's rollout of the same fields (2 and 10 aircraft; and a horizon
    shorter than the steps the fields cover)."""
    import torch
    horizon = None
    if which == "c1":
        s = _ar1(synth.c1, prec, M=4, grid=(8, 8, 4))
    else:
        s = _ar1(synth.c2, prec, M=4, grid=(8, 8, 4), H=90, S=6)
        if which == "c2-short":
            horizon = 61
    ctx = lib.smc_mpc_init(s)
    P, N, M = 96, s["N"], s["M"]
    rnp = np.float64 if prec == "fp64" else np.float32
    u = np.random.default_rng(5).uniform(0, 1, (P, N, s["S"], 3)).astype(rnp).astype(np.float64)
    W = owind.sample_field(s, 2).astype(rnp).astype(np.float64)       # [H, M, G, 2]
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    steps = zeros((128,), torch.int64)
    H = s["H"] if horizon is None else horizon
    lib.smc_k_rollout(ctx, dev(u, ctx.real_dtype), P, dev(W, ctx.real_dtype), dev(s["states"]),
                      dev(np.asarray(s["k_active"], np.int32)), H, cost, feas, steps)
    ref = oro.rollout(s, u, W, horizon=H, with_margins=True)
    got_c = host(cost).transpose(1, 0, 2)
    got_f = host(feas).transpose(1, 0, 2).astype(bool)
    cnt = host(steps)
    assert int(cnt[:64].sum()) == ref["steps"] and int(cnt[64:].sum()) == ref["pair_tests"]
    near = 1e-9 if prec == "fp64" else 1e-4
    ok = ~np.broadcast_to((ref["margin"] < near).any(axis=2, keepdims=True), ref["margin"].shape)
    assert ok.mean() > 0.8
    assert np.all(got_f[ok] == ref["feas"][ok])
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert rel_err(got_c, ref["cost"])[ok].max() < tol


@pytest.mark.parametrize("move", ["jitter", "rwmh"])
def test_c1_step_with_time_correlated_wind_matches_oracle(lib, move):
    """A whole FP64 MPC update under the paper's wind model returns the
    oracle's particle, controls within 1e-4 and cost within 1e-5."""
    s = synth.shrink(synth.c1(wind_model="ar1", move=move), L=128, K=8)
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    assert status == (1 if ref["infeasible"] else 0)
    assert info["best_particle"] == ref["best"]
    assert np.abs((ctrl - lo) / (hi - lo) - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_eval_cost_with_time_correlated_wind(lib, prec):
    s = _ar1(synth.c2, prec, M=5, grid=(8, 8, 4), H=60, S=6)
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(9)
    parts = rng.uniform(0, 1, (17, s["N"], s["S"], 3))
    if prec == "fp32":
        parts = parts.astype(np.float32).astype(np.float64)
    cost, feas = lib.smc_eval_cost(ctx, parts, 4)
    rc, rf = osmc.eval_cost(s, parts, 4)
    ok = feas == rf
    assert ok.mean() > 0.9
    assert np.all(rel_err(cost, rc)[ok] < (1e-6 if prec == "fp64" else 2e-5))


def test_time_correlated_wind_rejects_unsupported_calls(lib):
    import torch
    s = _ar1(synth.c1, M=2, grid=(4, 4, 2), L=16)
    ctx = lib.smc_mpc_init(s)
    with pytest.raises(lib.SmcError):
        lib.smc_set_rollout_layout(ctx, 1)
    P, N = 4, s["N"]
    u = zeros((P, N, s["S"], 3), torch.float64)
    W = zeros((s["H"], 2, 32, 2), torch.float64)
    g = zeros((P, N, s["S"], 3), torch.float64)
    with pytest.raises(lib.SmcError):
        lib.smc_k_rollout_grad(ctx, u, P, W, dev(s["states"]),
                               dev(np.asarray(s["k_active"], np.int32)), s["H"], g)


def test_full_size_c2_fields_and_rollout_sampled(lib):
    """C2 at full size under the paper's wind (8192 particles x 64 samples x
    10 aircraft x 120 steps; 120 x 64 fields of 8192 points), the launches
    the benchmark times: the GPU's fields of two samples against the
    oracle's recursion for those samples (normals drawn by the oracle from
    their counters), then 24 worlds of those samples, rolled out on the
    GPU's own fields, against the oracle's rollout on the oracle's fields."""
    import torch
    from oracle import philox
    s = synth.c2(wind_model="ar1")
    ctx = lib.smc_mpc_init(s)
    P, M, N, S, H = s["L"], s["M"], s["N"], s["S"], s["H"]
    G, J = ctx.G, 5
    W = empty((H, M, G, 2), torch.float32)
    lib.smc_k_wind_fields(ctx, s["mpc_step"], J, s["wind_mean"], W)
    rng = np.random.default_rng(21)
    u = rng.uniform(0, 1, (P, N, S, 3)).astype(np.float32)
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    lib.smc_k_rollout(ctx, dev(u), P, W, dev(s["states"]), dev(np.asarray(s["k_active"], np.int32)),
                      H, cost, feas)
    gc, gf, Wg = host(cost), host(feas).astype(bool), host(W)
    Q = owind.factor(s)
    a = owind.ar1_coefficient(s["dt"], s["wind_tcorr"])
    ax, ay, az = owind.grid_axes(s["box"], s["grid"])
    kap = (np.linalg.cond(owind.exp_gram_h(ax, ay, s["wind_beta"]) + s["wind_nugget"] * np.eye(len(ax) * len(ay)))
           + np.linalg.cond(owind.exp_gram_z(az, s["wind_gamma"]) + s["wind_nugget"] * np.eye(len(az))))
    u32 = 2.0 ** -24
    compared = 0
    for m in (0, M - 1):
        e = ((np.arange(H, dtype=np.int64)[:, None] * M + m) * G
             + np.arange(G, dtype=np.int64)[None, :]).reshape(-1)
        z0, z1 = philox.normals_pair(s["seed"], s["mpc_step"], J, philox.WIND, e, 0)
        V = np.stack([z0.reshape(H, G), z1.reshape(H, G)], axis=-1)[:, :, None, :]
        Wo = owind.ar1_fields(Q, V, a, s["wind_mean"])                     # [H, 1, G, 2]
        bound = _field_bound(Q, V, a).transpose(0, 2, 1, 3)
        tol = (2 * u32 * (4 + np.sqrt(G) + H) + 4 * 2.0 ** -53 * kap) * bound + u32 * np.abs(Wo)
        err = np.abs(Wg[:, m:m + 1].astype(np.float64) - Wo)
        assert np.all(err <= tol), (m, err.max())
        for p in rng.integers(P, size=12):
            r = oro.rollout(s, u[p:p + 1].astype(np.float64), Wo, with_margins=True)
            if (r["margin"] < 1e-4).any():
                continue
            compared += 1
            assert np.array_equal(gf[m, p], r["feas"][0, 0]), (p, m)
            assert np.all(rel_err(gc[m, p], r["cost"][0, 0]) < 2e-5), (p, m)
    assert compared >= 16


@pytest.mark.parametrize("grid", [(6, 5, 3), (8, 8, 4)])
def test_frozen_time_correlation_repeats_the_first_field(lib, grid):
    """G_t = infinity: a = 1 and Q = 0, so every step's field is the first
    one bit for bit (both the two-pass and the fused normals kernels), and
    the first is the oracle's."""
    import math
    s = _ar1(synth.c1, "fp32", grid=grid, M=3, H=10, S=5)
    s["wind_tcorr"] = math.inf
    ctx = lib.smc_mpc_init(s)
    W = empty((10, 3, ctx.G, 2), ctx.real_dtype)
    lib.smc_k_wind_fields(ctx, 0, 2, s["wind_mean"], W)
    got = host(W)
    for k in range(1, 10):
        assert np.array_equal(got[k], got[0]), k
    ref = owind.sample_field(s, 2)
    assert np.abs(got[0] - ref[0]).max() < 1e-4 * s["wind_sigma"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_steps", [1, 12])
def test_plant_step_time_correlated_wind_matches_oracle(lib, prec, n_steps):
    """The plant under the paper's wind model flies sample 0's field of each
    step (iteration word plant_iter): ten aircraft, random plans; states,
    activation steps and events against the oracle's plant."""
    import math
    s = _ar1(synth.c2, prec, M=4, L=8, K=2, H=30, S=3, grid=(8, 8, 4))
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(n_steps)
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    ctrl = lo + rng.uniform(0.2, 0.8, (s["N"], s["S"], 3)) * (hi - lo)
    from oracle import mpc as ompc
    got = lib.smc_plant_step(ctx, ctrl, plant_iter=5, n_steps=n_steps, mpc_step=3)
    ref = ompc.plant_step(s, ctrl, s["states"], s["k_active"], n_steps, plant_iter=5, mpc_step=3)
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    scale = np.array([1e5, 1e5, 1e4, 250.0, 2 * math.pi, 1e5])
    assert (np.abs(got[0] - ref[0]) / scale).max() < tol


def test_rolling_window_time_correlated_wind_matches_oracle(lib):
    """Two receding-horizon updates of C1 in FP64 under the paper's wind
    model, the plant flying sample 0's step fields: the oracle's controls,
    plant states, activation steps and events."""
    from oracle import mpc as ompc
    s = _ar1(synth.c1, L=64, K=4)
    got = lib.rolling_window(lib.smc_mpc_init(s), 2)
    ref = ompc.rolling_window(s, 2)
    for t, (g, r) in enumerate(zip(got, ref)):
        assert np.abs(g["controls"] - r["controls"]).max() < 1e-6 * 250.0, t
        assert np.array_equal(g["k_active"], r["k_active"]) and np.array_equal(g["event"], r["event"])
        assert np.all(rel_err(g["states"], r["states"], floor=1.0) < 1e-8), t
