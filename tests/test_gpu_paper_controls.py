"""GPU parity of the paper's own control parametrisation (per-step thrust,
flight-path angle and bank; Sec. "Trajectory Planning and Disturbance
Realisations", eq. hor) in the world-per-lane rollout: element-wise against
the FP64 oracle in both precisions, whole FP64 updates against the oracle's
(tempered and the paper's literal weighting), and the refused
combinations."""
import numpy as np
import pytest

import synth
from oracle import smc as osmc
from tests.test_gpu_kernels import _compare_rollout, _rollout_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("N", [2, 10, 20])
def test_rollout_paper_controls(lib, prec, N):
    n_arr = max(1, (3 * N) // 5)
    s = synth.make_scenario("T", n_arr=n_arr, n_dep=N - n_arr, box=(80e3, 80e3, 6e3),
                            grid=(6, 5, 4), H=24, dt=5.0, S=24, M=5, L=8, K=2,
                            precision=prec, controls="paper", seed=N, dep_spacing=3)
    assert s["S"] == s["H"] == 24 and s["control_model"] == 1
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=37, seed=N)
    n_near = _compare_rollout(gc, gf, ref, s["precision"])
    assert steps == ref["steps"]
    assert n_near <= 0.05 * 37 * 5 + 2 * 5


def test_rollout_paper_controls_short_horizon(lib):
    """A rolling-window horizon below horizon_max: step k still takes
    control set k."""
    s = synth.make_scenario("T", n_arr=3, n_dep=1, box=(80e3, 80e3, 6e3), grid=(4, 4, 3),
                            H=20, dt=5.0, S=20, M=3, L=8, K=2, precision="fp64",
                            controls="paper", seed=7)
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=19, seed=3, horizon=13)
    _compare_rollout(gc, gf, ref, 0)
    assert steps == ref["steps"]


@pytest.mark.parametrize("move", ["jitter", "rwmh"])
def test_c1_paper_controls_step_matches_oracle(lib, move):
    s = synth.shrink(synth.c1(controls="paper", move=move), L=128, K=6)
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    assert info["best_particle"] == ref["best"]
    u = (ctrl - s["ctrl_lo"]) / (s["ctrl_hi"] - s["ctrl_lo"])
    assert np.abs(u - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)


def test_paper_table_shape_with_literal_weighting_matches_oracle(lib):
    """The paper's timing workload shape (10 aircraft, horizon 6 of 10 s,
    per-step controls, literal weighting over SampleSchedule(J) + 1 passes)
    shrunk to 256 particles and 5 iterations, in FP64."""
    s = synth.shrink(synth.paper_table(K=5, precision="fp64"), L=256)
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    assert info["best_particle"] == ref["best"]
    u = (ctrl - s["ctrl_lo"]) / (s["ctrl_hi"] - s["ctrl_lo"])
    assert np.abs(u - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)


def test_paper_controls_refusals(lib):
    s = synth.shrink(synth.c1(controls="paper"), L=16, K=2)
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_init(dict(s, move=2))                          # no adjoint
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_init(dict(s, S=s["H"] - 1))                    # a control set per step
    ctx = lib.smc_mpc_init(s)
    for layout in (1, 3):
        with pytest.raises(lib.SmcError):
            lib.smc_set_rollout_layout(ctx, layout)
    with pytest.raises(lib.SmcError):
        lib.smc_plant_step(ctx, np.full((s["N"], s["S"], 3), 0.5), 0, n_steps=1)
