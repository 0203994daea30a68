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


@pytest.mark.parametrize("M", [1, 9, 16])
def test_reduce_product_matches_oracle(lib, M):
    """The literal weights of random passes (with violations and a zero
    objective) against the oracle's, element by element."""
    import torch
    from tests.gpu_helpers import dev, empty, host
    s = synth.c1()
    ctx = lib.smc_mpc_init(s)
    P, N = 301, s["N"]
    rng = np.random.default_rng(M)
    cost = rng.uniform(0, 1, (M, P, N))
    cost[0, 5, 0] = 1.0
    feas = rng.uniform(size=(M, P, N)) > 0.01
    chat = empty((P, N), torch.float64)
    fpn = empty((P, N), torch.uint8)
    logw = empty((P, N), torch.float64)
    lib.smc_k_reduce_product(ctx, P, M, dev(cost), dev(feas.astype(np.uint8)), chat, fpn, logw)
    c_t, f_t = cost.transpose(1, 0, 2), feas.transpose(1, 0, 2)
    rc, rf = osmc.expected_cost(c_t, f_t)
    rl = osmc.product_log_weights(c_t, f_t)
    gl = host(logw)
    assert np.abs(host(chat) - rc).max() < 4e-16
    assert np.array_equal(host(fpn).astype(bool), rf)
    assert gl[5, 0] == -np.inf
    assert np.array_equal(np.isfinite(gl), np.isfinite(rl))
    fin = np.isfinite(rl)
    assert np.all(np.abs(gl[fin] - rl[fin]) <= 1e-14 * np.maximum(np.abs(rl[fin]), 1.0))
    # more passes than the context's samples: refused by the library (the
    # buffers are sized for them, so the binding's size checks pass)
    big = np.zeros((s["M"] + 1,) + cost.shape[1:])
    with pytest.raises(lib.SmcError):
        lib.smc_k_reduce_product(ctx, P, s["M"] + 1, dev(big), dev(big.astype(np.uint8)),
                                 chat, fpn, logw)
