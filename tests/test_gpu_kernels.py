"""GPU parity of each hot-path kernel against the FP64 oracle, on identical
inputs, through the C ABI.

Tolerances:
  * integer work (Philox words, ancestors, selection index): bit-exact;
  * FP64 kernels: a few ulps of the operation count involved (Box-Muller and
    trilinear/dynamics transcendentals differ by libm/ocml ulps);
  * FP32 kernels: 1e-5 relative on per-particle expected cost, as the
    target states, with near-threshold decisions (relative margin < 1e-4)
    excluded and counted.
"""
import math

import numpy as np
import pytest

import synth
from oracle import philox as oph
from oracle import rollout as oro
from oracle import smc as osmc
from oracle import wind as owind
from tests.gpu_helpers import dev, empty, host, rel_err, separable_field, small_scenario, zeros

pytestmark = pytest.mark.gpu


def _ctx(lib, scen):
    return lib.smc_mpc_init(scen)


# ---- RNG -------------------------------------------------------------------------

@pytest.mark.parametrize("stream", [(0, 0, 0, 1, 0), (123456789012345, 7, 3, 2, 5),
                                    (2**64 - 1, -1, 2**31 - 1, 6, 255)])
def test_philox_words_bit_exact(lib, stream):
    import torch
    seed, step, J, purpose, scen = stream
    for e0, n in ((0, 1), (0, 1000), (2**32 - 5, 5), (77777, 4097)):
        out = zeros((n, 4), torch.int32)
        lib.smc_k_philox(seed, step, J, purpose, scen, e0, n, out)
        got = host(out).view(np.uint32)
        ref = oph.words(seed, step, J, purpose, np.arange(e0, e0 + n, dtype=np.int64), scen)
        assert np.array_equal(got, np.stack(ref, axis=1))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_init_particles(lib, prec):
    s = small_scenario("c1", prec)
    ctx = _ctx(lib, s)
    P = 300
    u = empty((P, s["N"], s["S"], 3), ctx.real_dtype)
    lib.smc_k_init_particles(ctx, 5, P, u)
    ref = osmc.init_particles(s, mpc_step=5, L=P)
    got = host(u)
    if prec == "fp64":
        assert np.array_equal(got, ref)
    else:
        assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wind_normals(lib, prec):
    s = small_scenario("c1", prec)
    ctx = _ctx(lib, s)
    G, M = ctx.G, ctx.M
    Z = empty((G, 2 * M), ctx.real_dtype)
    lib.smc_k_wind_normals(ctx, 2, 9, Z)
    ref = owind.wind_normals(s["seed"], 2, 9, G, M).reshape(G, 2 * M)
    got = host(Z).astype(np.float64)
    if prec == "fp64":
        assert np.abs(got - ref).max() < 1e-13
    else:
        assert np.abs(got - ref).max() < 6e-7 * max(1.0, np.abs(ref).max())


def test_wind_factor_matches_kronecker(lib):
    s = small_scenario("c1", "fp64")
    ctx = _ctx(lib, s)
    out = empty((ctx.G, ctx.G), ctx.real_dtype)
    lib.smc_k_wind_factor(ctx, out)
    ref = owind.kron_factor(s["box"], s["grid"], s["wind_sigma"], s["wind_ell"], s["wind_nugget"])
    # The two sides factor each axis in their own operation order (the
    # library row by row on the host, the oracle through LAPACK).  To first
    # order a Cholesky factor of a matrix with condition number kappa moves
    # by u kappa under rounding, and every factor entry is at most 1, so an
    # entry of sigma Lx (x) Ly (x) Lz moves by at most sigma u sum_a kappa_a
    # (with a factor 4 of slack), plus the rounding of the two products.
    u = 2.0 ** -53
    ax, ay, az = owind.grid_axes(s["box"], s["grid"])
    kap = sum(np.linalg.cond(owind.se_gram(a, s["wind_ell"]) + s["wind_nugget"] * np.eye(len(a)))
              for a in (ax, ay, az))
    tol = s["wind_sigma"] * 4 * u * kap + 4 * u * np.abs(ref)
    err = np.abs(host(out) - ref)
    assert np.all(err <= tol), (err.max(), (err / tol).max())


# up to 16 levels: the grouped product (levels' factor, then the horizontal
# factor's GEMM); 17 levels: the dense factor's GEMM
@pytest.mark.parametrize("prec,grid,M", [("fp64", (16, 16, 4), 16), ("fp64", (5, 7, 3), 3),
                                         ("fp32", (16, 16, 4), 16), ("fp32", (32, 32, 8), 64),
                                         ("fp32", (9, 6, 5), 40), ("fp64", (4, 5, 17), 6),
                                         ("fp32", (4, 5, 17), 6)])
def test_wind_gemm(lib, prec, grid, M):
    s = synth.shrink(small_scenario("c1", prec), grid=grid, M=M)
    ctx = _ctx(lib, s)
    G = ctx.G
    rng = np.random.default_rng(G + M)
    Zr = rng.standard_normal((G, 2 * M))
    if prec == "fp32":
        Zr = Zr.astype(np.float32).astype(np.float64)
    Lf = owind.kron_factor(s["box"], s["grid"], s["wind_sigma"], s["wind_ell"], s["wind_nugget"])
    wm = np.array([1.5, -2.0])
    ref = owind.wind_field(Lf, Zr.reshape(G, M, 2), wm)
    W = empty((M, G, 2), ctx.real_dtype)
    lib.smc_k_wind_gemm(ctx, dev(Zr, ctx.real_dtype), wm, W)
    got = host(W).astype(np.float64)
    # rounding of a G-term dot product: |error| <~ u sqrt(G) sum|L||Z| for
    # random-signed partial sums (u = unit roundoff) and of the output, on
    # top of the difference of the two factors: the library's host Cholesky
    # and the oracle's LAPACK one differ by their first-order rounding
    # sensitivity u kappa (bounded by test_wind_factor_matches_kronecker), and
    # in FP32 the factor is also rounded to FP32; that adds |dL| |Z|
    Lg = empty((G, G), ctx.real_dtype)
    lib.smc_k_wind_factor(ctx, Lg)
    dL = np.abs(host(Lg).astype(np.float64) - Lf)
    del Lg
    ax, ay, az = owind.grid_axes(s["box"], s["grid"])
    kap = sum(np.linalg.cond(owind.se_gram(a, s["wind_ell"]) + s["wind_nugget"] * np.eye(len(a)))
              for a in (ax, ay, az))
    u_f = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24   # rounding of the stored factor
    assert np.all(dL <= s["wind_sigma"] * 4 * 2.0 ** -53 * kap + 4 * u_f * np.abs(Lf))
    factor_term = (dL @ np.abs(Zr)).max()
    scale = (np.abs(Lf) @ np.abs(Zr)).max()
    u = 2.0 ** -53 if prec == "fp64" else 2.0 ** -24
    err = np.abs(got - ref).max()
    assert err <= 2 * u * scale * (2 + np.sqrt(G)) + factor_term, (err, factor_term)


# ---- rollout ---------------------------------------------------------------------

def _rollout_case(lib, s, P, seed=0, horizon=None, states=None, k_active=None, u=None, W=None,
                  layout=0):
    import torch
    ctx = _ctx(lib, s)
    lib.smc_set_rollout_layout(ctx, layout)
    rng = np.random.default_rng(seed)
    N, S, M = s["N"], s["S"], s["M"]
    H = s["H"] if horizon is None else horizon
    states = s["states"] if states is None else states
    k_active = s["k_active"] if k_active is None else k_active
    if u is None:
        u = rng.uniform(0, 1, (P, N, S, 3))
    if W is None:
        W = separable_field(s, seed + 100)
    rnp = np.float64 if s["precision"] == 0 else np.float32
    u = u.astype(rnp).astype(np.float64)
    W = W.astype(rnp).astype(np.float64)
    cost = empty((M, P, N), torch.float64)
    feas = empty((M, P, N), torch.uint8)
    steps = zeros((128,), torch.int64)
    lib.smc_k_rollout(ctx, dev(u, ctx.real_dtype), P, dev(W, ctx.real_dtype), dev(states),
                      dev(np.asarray(k_active, np.int32)), H, cost, feas, steps)
    ref = oro.rollout(s, u, W, states, k_active, H, with_margins=True)
    got_c = host(cost).transpose(1, 0, 2)
    got_f = host(feas).transpose(1, 0, 2).astype(bool)
    cnt = host(steps)
    assert int(cnt[64:].sum()) == ref["pair_tests"]
    return ctx, got_c, got_f, int(cnt[:64].sum()), ref


def _compare_rollout(got_c, got_f, ref, prec, near=None):
    near = (1e-9 if prec == 0 else 1e-4) if near is None else near
    margin = ref["margin"]
    # a world with any near-threshold decision may legitimately differ
    world_near = (margin < near).any(axis=2, keepdims=True) | (margin < near)
    world_near = np.broadcast_to(world_near.any(axis=2, keepdims=True), margin.shape)
    ok = ~world_near
    tol = 1e-10 if prec == 0 else 2e-5
    err = rel_err(got_c, ref["cost"])
    assert np.all(got_f[ok] == ref["feas"][ok])
    assert err[ok].max() < tol, err[ok].max()
    return int(world_near[..., 0].sum())


LAYOUTS = [1, 2]   # aircraft-per-lane, world-per-lane


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rollout_c1_shape(lib, prec, layout):
    s = small_scenario("c1", prec)
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=200, layout=layout)
    n_near = _compare_rollout(gc, gf, ref, s["precision"])
    assert steps == ref["steps"]
    assert n_near < 0.05 * 200 * s["M"]
    # per-particle expected cost (mean over samples)
    chat_ref, _ = osmc.expected_cost(ref["cost"], ref["feas"])
    world_near = (ref["margin"] < (1e-9 if prec == "fp64" else 1e-4)).any(axis=(1, 2))
    err = rel_err(gc.mean(axis=1), chat_ref)[~world_near]
    assert err.max() < (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rollout_c2_shape_ragged(lib, prec, layout):
    """10 aircraft (worlds of 10 lanes, 6 per wave, 4 idle lanes), staggered
    departures, P not a multiple of the worlds per wave, grid 32x32x8."""
    s = synth.shrink(synth.c2(precision=prec), M=5)
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=37, seed=4, layout=layout)
    n_near = _compare_rollout(gc, gf, ref, s["precision"])
    assert steps == ref["steps"]
    assert n_near < 0.25 * 37 * 5


@pytest.mark.parametrize("N,layout", [(1, 1), (2, 1), (3, 1), (7, 1), (16, 1), (24, 1), (33, 1),
                                      (40, 1), (48, 1), (63, 1), (64, 1),
                                      (1, 2), (2, 2), (3, 2), (5, 2), (7, 2), (9, 2), (10, 2),
                                      (11, 2), (13, 2), (16, 2)])
def test_rollout_aircraft_counts(lib, N, layout):
    """Worlds from 1 lane to a full wave; mixed kinds and activation steps.
    33 .. 63 aircraft use the packed aircraft-per-lane layout (worlds across
    wavefronts of a workgroup)."""
    rng = np.random.default_rng(N)
    n_arr = min(max(1, N // 2), 12)
    s = synth.make_scenario("T", n_arr=n_arr, n_dep=N - n_arr,
                            box=(100e3, 100e3, 8e3), grid=(6, 5, 4), H=30, dt=5.0, S=3,
                            M=3, L=8, K=2, precision="fp64", seed=N)
    k_act = s["k_active"].copy()
    k_act[rng.uniform(size=N) < 0.2] = -1
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=11, seed=N, horizon=27, k_active=k_act,
                                            layout=layout)
    _compare_rollout(gc, gf, ref, 0)
    assert steps == ref["steps"]


@pytest.mark.parametrize("N,layout", [(12, 1), (12, 2), (40, 1), (41, 1)])
def test_rollout_close_traffic_separation(lib, N, layout):
    """Aircraft packed inside one separation cell so that many pair tests
    fire, exercising both the pair split and the mask reduction (40 and 41
    aircraft: the packed layout, even and odd pair split)."""
    rng = np.random.default_rng(5)
    s = synth.make_scenario("T", n_arr=0, n_dep=N, box=(60e3, 60e3, 6e3), grid=(4, 4, 3),
                            H=8, dt=5.0, S=2, M=2, L=4, K=2, precision="fp64", seed=1)
    st = np.zeros((N, 6))
    st[:, 0] = rng.uniform(-8e3, 8e3, N)
    st[:, 1] = rng.uniform(-8e3, 8e3, N)
    st[:, 2] = rng.uniform(2000, 2800, N)
    st[:, 3] = 150.0
    st[:, 4] = rng.uniform(-3, 3, N)
    st[:, 5] = 60e3
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=50, states=st, k_active=np.zeros(N, np.int32),
                                            layout=layout)
    _compare_rollout(gc, gf, ref, 0)
    assert (~ref["feas"]).mean() > 0.2


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_rollout_landed_aircraft_leave_the_airspace(lib, prec, layout):
    """Arrivals queued on the final approach 6.5 km apart at one altitude:
    each lands where the one before it landed.  A landed aircraft no longer
    takes part in separation (Sec. "Constraint Handling"), so no world may
    report a conflict; any residual presence of landed aircraft would make
    every world infeasible."""
    n, H = 4, 40
    s = synth.make_scenario("Q", n_arr=n, n_dep=0, box=(80e3, 80e3, 6e3), grid=(4, 4, 3),
                            H=H, dt=5.0, S=4, M=2, L=4, K=2, precision=prec, seed=3)
    s = dict(s)
    s["ctrl_lo"] = np.array([-0.1 * np.pi / 180, 110.0, -0.5])
    s["ctrl_hi"] = np.array([0.1 * np.pi / 180, 128.0, 0.5])
    st = np.zeros((n, 6))
    st[:, 0] = 8.3e3 + 6.5e3 * np.arange(n)
    st[:, 2] = 500.0
    st[:, 3] = 120.0
    st[:, 4] = np.pi
    st[:, 5] = 60e3
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=64, states=st,
                                            k_active=np.zeros(n, np.int32), layout=layout)
    _compare_rollout(gc, gf, ref, s["precision"])
    assert steps == ref["steps"] < 64 * 2 * n * H        # aircraft did land
    assert ref["feas"].all() and gf.all()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rollout_noise_term(lib, layout):
    s = synth.shrink(synth.c5(precision="fp64"), M=2, H=30, S=3, grid=(8, 8, 4))
    s = dict(s)
    keep = [0, 1, 2, 24, 25]
    for k in ("kind", "aircraft", "targets", "states", "k_active"):
        s[k] = s[k][keep]
    s["N"] = len(keep)
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=20, layout=layout)
    _compare_rollout(gc, gf, ref, 0)


# ---- weights, resampling, moves, selection -------------------------------------

def test_reduce_matches_oracle(lib):
    import torch
    s = small_scenario("c1", "fp64")
    ctx = _ctx(lib, s)
    P, M, N = 97, s["M"], s["N"]
    rng = np.random.default_rng(0)
    cost = rng.uniform(0, 1, (M, P, N))
    feas = rng.uniform(size=(M, P, N)) > 0.02
    chat = empty((P, N), torch.float64)
    fpn = empty((P, N), torch.uint8)
    logw = empty((P, N), torch.float64)
    lib.smc_k_reduce(ctx, P, dev(cost), dev(feas.astype(np.uint8)), 8.0, chat, fpn, logw)
    rc, rf = osmc.expected_cost(cost.transpose(1, 0, 2), feas.transpose(1, 0, 2))
    assert np.abs(host(chat) - rc).max() < 4e-16
    assert np.array_equal(host(fpn).astype(bool), rf)
    rl = osmc.log_weights(rc, rf, 8.0)
    gl = host(logw)
    assert np.array_equal(np.isfinite(gl), np.isfinite(rl))
    assert np.abs(gl[np.isfinite(rl)] - rl[np.isfinite(rl)]).max() < 1e-14


@pytest.mark.parametrize("P", [1, 2, 7, 256, 1000, 1025, 8192, 65536])
def test_resample_bit_exact(lib, P):
    import torch
    N = 3
    s = synth.shrink(small_scenario("c1", "fp64"), L=max(P, 2))
    s = dict(s)
    for k in ("kind", "aircraft", "targets", "states", "k_active"):
        s[k] = np.concatenate([s[k], s[k][:1]])
    s["N"] = N
    ctx = _ctx(lib, s)
    rng = np.random.default_rng(P)
    logw = rng.normal(0, 4, (P, N)) - 30.0
    logw[rng.uniform(size=(P, N)) < 0.3] = -np.inf
    logw[:, 2] = -np.inf                   # an all-violating row
    if P > 1:
        logw[0, 0] = -30.0                 # keep row 0 non-empty
    U = rng.integers(0, 2**32, N, dtype=np.uint64).astype(np.uint32)
    anc = empty((N, P), torch.int32)
    lib.smc_k_resample(ctx, P, dev(logw), dev(U.view(np.int32)), anc)
    got = host(anc)
    for i in range(N):
        ref = osmc.resample_row(logw[:, i], int(U[i]))
        assert np.array_equal(got[i], ref), i


def test_resample_offsets_and_gather_jitter(lib):
    import torch
    s = small_scenario("c1", "fp64")
    ctx = _ctx(lib, s)
    N, S, P = s["N"], s["S"], 333
    U = empty((N,), torch.int32)
    lib.smc_k_resample_offsets(ctx, 4, 6, U)
    assert [int(x) for x in host(U).view(np.uint32)] == osmc.resample_offsets(s, 6, N, 4)
    rng = np.random.default_rng(1)
    u = rng.uniform(0, 1, (P, N, S, 3))
    anc = np.sort(rng.integers(0, P, (N, P)), axis=1).astype(np.int32)
    out = empty((P, N, S, 3), torch.float64)
    for jit in (0, 1):
        lib.smc_k_gather_move(ctx, P, dev(u), dev(anc), out, 4, 6, jit)
        ref = osmc.gather(u, anc)
        if jit:
            ref = osmc.jitter(s, ref, 6, mpc_step=4)
        assert np.abs(host(out) - ref).max() < 1e-15


def test_propose_accept_select(lib):
    import torch
    s = small_scenario("c1", "fp64")
    s = dict(s, move=1)
    ctx = _ctx(lib, s)
    N, S, P = s["N"], s["S"], 257
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 1, (P, N, S, 3))
    up = empty((P, N, S, 3), torch.float64)
    lib.smc_k_propose(ctx, P, dev(u), up, 3, 5)
    ref_up = osmc.rw_propose(s, u, 5, mpc_step=3)
    assert np.abs(host(up) - ref_up).max() < 1e-15
    chat = rng.uniform(0, 1, (P, N))
    chat2 = rng.uniform(0, 1, (P, N))
    f1 = rng.uniform(size=(P, N)) > 0.1
    f2 = rng.uniform(size=(P, N)) > 0.1
    l1 = osmc.log_weights(chat, f1, 9.0)
    l2 = osmc.log_weights(chat2, f2, 9.0)
    acc_ref = osmc.mh_accept(s, 5, l1, l2, mpc_step=3)
    d_u, d_chat, d_f, d_l = dev(u), dev(chat), dev(f1.astype(np.uint8)), dev(l1)
    acc = empty((P,), torch.int32)
    lib.smc_k_accept(ctx, P, d_u, dev(ref_up), d_chat, dev(chat2), d_f,
                     dev(f2.astype(np.uint8)), d_l, dev(l2), 3, 5, acc)
    assert np.array_equal(host(acc).astype(bool), acc_ref)
    assert np.array_equal(host(d_u), np.where(acc_ref[:, None, None, None], ref_up, u))
    assert np.array_equal(host(d_chat), np.where(acc_ref[:, None], chat2, chat))
    # selection
    lw = np.where(acc_ref[:, None], l2, l1)
    ch = np.where(acc_ref[:, None], chat2, chat)
    best = empty((2,), torch.int32)
    lib.smc_k_select(ctx, P, dev(lw), dev(ch), 9.0, best)
    l_ref, bad = osmc.select_best(lw, ch, 9.0)
    assert list(host(best)) == [l_ref, int(bad)]
    # all infeasible -> fewest violators, then cost
    lw2 = lw.copy()
    lw2[:, 0] = -np.inf
    lib.smc_k_select(ctx, P, dev(lw2), dev(ch), 9.0, best)
    l_ref, bad = osmc.select_best(lw2, ch, 9.0)
    assert list(host(best)) == [l_ref, 1]
    # exact ties -> lowest index
    lw3 = np.full((P, N), -1.0)
    ch3 = np.full((P, N), 1.0 / 9.0)
    lib.smc_k_select(ctx, P, dev(lw3), dev(ch3), 9.0, best)
    assert list(host(best)) == [0, 0]
