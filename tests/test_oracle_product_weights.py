"""Pins of the oracle's literal weighting (Alg. 1 inner loop; Sec. "Weight
Scaling"; Sec. "Simulation Setup" for the schedule): S(J) + 1 passes at
iteration J, each multiplying the weight by the objective value 1 - cost,
any violation zeroing it."""
import math

import numpy as np

import synth
from oracle import smc


def test_inner_passes_follow_the_schedule():
    # j runs from 0 while j <= floor(3 + 5 e^{0.05 J})
    assert [smc.inner_samples(J) for J in (0, 1, 20, 39)] == [9, 9, 17, 39]


def test_constant_cost_gives_the_power():
    """n passes at the same cost c: W = (1 - c)^n (up to 1/L)."""
    cost = np.full((3, 7, 2), 0.25)
    cost[1, :, 0] = 0.5
    feas = np.ones_like(cost, dtype=bool)
    lw = smc.product_log_weights(cost, feas)
    assert np.allclose(lw[0], 7 * math.log(0.75), rtol=1e-15, atol=0)
    assert lw[1, 0] == 7 * math.log(0.5)
    # the product over passes in any order: a permutation changes nothing
    rng = np.random.default_rng(0)
    c = rng.uniform(0, 0.9, (2, 9, 3))
    lw1 = smc.product_log_weights(c, np.ones_like(c, dtype=bool))
    lw2 = smc.product_log_weights(c[:, ::-1], np.ones_like(c, dtype=bool))
    assert np.array_equal(lw1, lw2)
    ref = np.log(np.prod(1.0 - c, axis=1))
    assert np.allclose(lw1, ref, rtol=1e-13, atol=0)


def test_violation_or_zero_objective_zeroes_the_weight():
    cost = np.full((2, 4, 2), 0.1)
    feas = np.ones_like(cost, dtype=bool)
    feas[0, 3, 1] = False          # one violating pass
    cost[1, 2, 0] = 1.0            # objective value 0 in one pass
    lw = smc.product_log_weights(cost, feas)
    assert lw[0, 1] == -np.inf and lw[1, 0] == -np.inf
    assert np.isfinite(lw[0, 0]) and np.isfinite(lw[1, 1])


def test_product_weighting_update_uses_the_first_samples():
    """An update with the literal weighting reads only the first S(J) + 1
    samples of each iteration: extra wind samples change nothing."""
    s = synth.shrink(synth.c1(), L=32, K=3, M=12, grid=(6, 6, 3))
    s["weighting"] = 1
    a = smc.smc_mpc_step(s)
    s2 = dict(s)
    s2["M"] = 16
    b = smc.smc_mpc_step(s2)
    assert a["best"] == b["best"] and a["cost"] == b["cost"]
    assert np.array_equal(a["u_best"], b["u_best"])
