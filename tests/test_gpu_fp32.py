"""The FP32 configuration (FP32 dynamics, FP64 weights and scans) against
the FP64 oracle over whole SMC iterations: a teacher-forced update, where
every iteration resamples with the oracle's ancestors so that the two runs
stay on one path, and the C2 workload's update against the FP64 path."""
import numpy as np
import pytest

import synth
from oracle import rollout as oro
from oracle import smc as osmc
from oracle import wind as owind
from tests.gpu_helpers import dev, empty, host, rel_err

pytestmark = pytest.mark.gpu


def test_teacher_forced_fp32_update_matches_oracle(lib):
    """Shrunk C2 (10 aircraft, L = 512, M = 16, K = 4, grid 16 x 16 x 4) in
    FP32.  Each iteration: the GPU draws its own normals and fields, rolls
    out and weighs its own particles; the oracle does the same in FP64 on
    its particles; then both gather with the oracle's ancestors and jitter.
    Per iteration: particles within 1e-6; every world (particle, sample)
    with no separation, landing or unary decision within 1e-4 (relative) of
    its threshold in the oracle has exact feasibility and costs within 1e-4,
    and at most 0.1 % of those worlds differ by more than 1e-5 (FP32
    positions carry errors of a few centimetres after 120 steps, and the
    geometric cost elements of an arrival a few kilometres from the runway
    amplify them to about 2e-5); a world whose cost differs more than 1e-4
    must be a near-threshold world;
    c_hat per (particle, aircraft) within 1e-5 relative for every particle
    whose worlds all agree (at least 90 % of them), and per-particle
    feasibility exact for particles with no near-threshold world.  (After
    resampling, copies of one ancestor share its near-threshold decisions,
    so a per-particle exclusion alone would leave few particles.)"""
    import torch
    s = synth.shrink(synth.c2(), L=512, K=4, M=16, grid=(16, 16, 4))
    assert s["precision"] == 1 and s["move"] == 0
    ctx = lib.smc_mpc_init(s)
    L, N, S, M, G, K, H = s["L"], s["N"], s["S"], s["M"], ctx.G, s["K"], s["H"]
    step = int(s["mpc_step"])
    f32 = torch.float32
    states, kact = dev(s["states"]), dev(np.asarray(s["k_active"], np.int32))
    u_ref = osmc.init_particles(s)
    u = empty((L, N, S, 3), f32)
    lib.smc_k_init_particles(ctx, step, L, u)
    Lfac = owind.factor(s)
    Z, W = empty((G, 2 * M), f32), empty((M, G, 2), f32)
    cost, feas = empty((M, L, N), torch.float64), empty((M, L, N), torch.uint8)
    chat, fpn, logw = (empty((L, N), torch.float64), empty((L, N), torch.uint8),
                       empty((L, N), torch.float64))
    u2 = empty((L, N, S, 3), f32)
    for J in range(K):
        assert np.abs(host(u).astype(np.float64) - u_ref).max() <= 1e-6, J
        b = osmc.beta(s, J)
        lib.smc_k_wind_normals(ctx, step, J, Z)
        lib.smc_k_wind_gemm(ctx, Z, s["wind_mean"], W)
        lib.smc_k_rollout(ctx, u, L, W, states, kact, H, cost, feas)
        lib.smc_k_reduce(ctx, L, cost, feas, b, chat, fpn, logw)
        r = oro.rollout(s, u_ref, owind.sample_field(s, J, step, Lfac), with_margins=True)
        c_ref, f_ref = osmc.expected_cost(r["cost"], r["feas"])
        gc = host(cost).transpose(1, 0, 2)                          # [L, M, N]
        gf = host(feas).transpose(1, 0, 2).astype(bool)
        world_near = (r["margin"] < 1e-4).any(axis=2)               # [L, M]
        err_w = rel_err(gc, r["cost"])
        assert np.array_equal(gf[~world_near], r["feas"][~world_near]), J
        off = err_w[~world_near]
        assert off.max() < 1e-4, (J, off.max())
        assert (off > 1e-5).mean() <= 1e-3, (J, float((off > 1e-5).mean()))
        flipped = (err_w > 1e-4).any(axis=2)                        # [L, M]
        assert not (flipped & ~world_near).any(), J
        agree = ~flipped.any(axis=1)                                # [L]
        assert agree.mean() >= 0.9, (J, float(agree.mean()))
        err = rel_err(host(chat), c_ref)[agree]
        assert err.max() < 1e-5, (J, err.max())
        near = world_near.any(axis=1)
        assert np.array_equal(host(fpn).astype(bool)[~near], f_ref[~near]), J
        if J == K - 1:
            break
        logw_ref = osmc.log_weights(c_ref, f_ref, b)
        anc = osmc.resample(logw_ref, osmc.resample_offsets(s, J, N))
        u_ref = osmc.jitter(s, osmc.gather(u_ref, anc), J)
        lib.smc_k_gather_move(ctx, L, u, dev(anc.astype(np.int32)), u2, step, J, 1)
        u, u2 = u2, u


def test_c2_fp32_update_against_fp64_path(lib):
    """The C2 workload (10 aircraft, L = 8192, M = 64, K = 40) in FP32 and in
    FP64 through smc_mpc_step, for three MPC steps (three draws of every
    random stream).  Once one resampling decision differs, the two updates
    are different Monte Carlo runs, so their returned costs differ by the
    run-to-run spread of the 40-iteration estimate (0.1 ... 0.8 % measured
    here, with either product of the wind fields): the FP32 path may not end
    worse than the FP64 path by more than 1 %, nor differ by more than 1 % on
    average.  What FP32 itself changes is checked exactly: the FP32 path's
    controls, re-scored by the FP64 path (smc_eval_cost on the last
    iteration's fields), cost what the FP32 path returned within 1e-4 (and the
    teacher-forced test above follows the iterations themselves)."""
    rel = []
    for step in (0, 1, 2):
        s32 = synth.c2()
        s64 = synth.c2(precision="fp64")
        s32["mpc_step"] = step
        s64["mpc_step"] = step
        c32 = lib.smc_mpc_init(s32)
        c64 = lib.smc_mpc_init(s64)
        ctrl32, cost32, st32, _ = lib.smc_mpc_step(c32)
        ctrl64, cost64, st64, _ = lib.smc_mpc_step(c64)
        assert st32 == st64 == 0
        assert cost32[0] <= cost64[0] * (1 + 1e-2), (step, cost32[0], cost64[0])
        rel.append(abs(cost32[0] - cost64[0]) / abs(cost64[0]))
        lo, hi = s64["ctrl_lo"], s64["ctrl_hi"]
        un = ((ctrl32 - lo) / (hi - lo))[None]
        rc, rf = lib.smc_eval_cost(c64, un, s64["K"] - 1)
        assert rf.all()
        assert abs(rc.sum() - cost32[0]) <= 1e-4 * abs(cost32[0]), (step, rc.sum(), cost32[0])
        c32.close()
        c64.close()
    assert np.mean(rel) <= 1e-2, rel
