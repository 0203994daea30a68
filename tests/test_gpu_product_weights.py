"""GPU parity of the paper's literal weighting (Alg. 1 inner loop; Sec.
"Weight Scaling"): SampleSchedule(J) + 1 passes per iteration, the weight
multiplied by the objective value of each; whole MPC updates against the
oracle's."""
import numpy as np
import pytest

import synth
from oracle import smc as osmc

pytestmark = pytest.mark.gpu


def _check(lib, s):
    ctx = lib.smc_mpc_init(s)
    ctrl, cost, status, info = lib.smc_mpc_step(ctx)
    ref = osmc.smc_mpc_step(s)
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    assert status == (1 if ref["infeasible"] else 0)
    assert info["best_particle"] == ref["best"]
    assert np.abs((ctrl - lo) / (hi - lo) - ref["u_best"]).max() < 1e-4
    assert abs(cost[0] - ref["cost"]) <= 1e-5 * max(abs(ref["cost"]), 1e-3)
    return info


@pytest.mark.parametrize("move", ["jitter", "rwmh"])
def test_c1_product_weighting_matches_oracle(lib, move):
    """C1 in FP64 (16 samples cover the 20 iterations' passes)."""
    s = synth.shrink(synth.c1(move=move), K=20 if move == "jitter" else 10)
    s["weighting"] = 1
    _check(lib, s)


def test_ten_aircraft_product_weighting_matches_oracle(lib):
    s = synth.shrink(synth.c2(precision="fp64"), L=256, M=12, K=8, grid=(8, 8, 4), H=60, S=6)
    s["weighting"] = 1
    info = _check(lib, s)
    # passes: sum over J of SampleSchedule(J) + 1 worlds per particle
    assert info["rollout_launches"] == 8


def test_product_weighting_limits(lib):
    s = synth.shrink(synth.c1(), K=20, M=15)     # SampleSchedule(19) + 1 = 16 passes
    s["weighting"] = 1
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_init(s)
    s = synth.shrink(synth.c1(move="mala"), K=4)
    s["weighting"] = 1
    with pytest.raises(lib.SmcError):
        lib.smc_mpc_init(s)
