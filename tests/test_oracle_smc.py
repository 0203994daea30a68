"""Pins of the oracle's SMC machinery (Alg. 1) on a separable toy quadratic
whose minimiser is known, plus the schedule and the final selection rule."""
import numpy as np
import pytest

from oracle import smc
from tests.oracle_helpers import mini


def _toy(move, L=512, K=40, N=3, S=2, seed=4):
    s = mini(N=N, S=S, L=L)
    s.update(K=K, move=move, seed=seed, kappa=1.0, sigma_move=0.02)
    rng = np.random.default_rng(9)
    target = rng.uniform(0.25, 0.75, (N, S, 3))
    A = rng.uniform(40.0, 120.0, (N, S * 3))

    def evaluate(u, J):
        d = (u - target[None]).reshape(u.shape[0], N, S * 3)
        return 0.5 * (A[None] * d * d).sum(-1), np.ones((u.shape[0], N), bool)

    res = smc.run_smc(s, evaluate, L, K, N, S)
    return res, target


@pytest.mark.parametrize("move", [0, 1])
def test_toy_quadratic_minimiser_recovered(move):
    res, target = _toy(move)
    best = res["u"][res["best"]]
    assert np.abs(best - target).max() < 0.06
    assert np.abs(res["u"].mean(0) - target).max() < 0.06
    if move == 1:
        assert 0.0 < np.mean(res["acc_rate"]) < 1.0


def test_schedule_values():
    vals = {0: 8, 19: 15, 39: 38, 59: 98, 100: 745}
    for J, v in vals.items():
        assert smc.sample_schedule(J) == v


def test_final_selection_rule():
    logw = np.array([[-1.0, -np.inf], [-2.0, -3.0], [-2.5, -2.5], [-0.1, -np.inf]])
    chat = -logw / 2.0
    chat[~np.isfinite(chat)] = 0.0
    l, bad = smc.select_best(logw, chat, 2.0)
    assert (l, bad) == (1, False)           # ties (-5 and -5): lowest index
    l, bad = smc.select_best(np.full((3, 2), -np.inf), np.array([[.3, .2], [.1, .1], [.1, .1]]), 1.0)
    assert (l, bad) == (1, True)


def test_jitter_stays_in_box_and_init_uniform():
    s = mini(N=2, S=3, L=4000)
    u = smc.init_particles(s)
    assert u.shape == (4000, 2, 3, 3) and u.min() > 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.01
    v = smc.jitter(s, u, 3)
    assert v.min() >= 0 and v.max() <= 1
    d = (v - u)[(v > 0) & (v < 1)]
    assert abs(d.std() - s["sigma_move"]) < 0.001
    r = smc.reflect(np.array([-0.25, 0.5, 1.25, 2.5, -1.5]))
    assert np.allclose(r, [0.25, 0.5, 0.75, 0.5, 0.5])


def test_toy_quadratic_mala():
    """Langevin moves with the exact toy gradient recover the minimiser."""
    s = mini(N=2, S=2, L=256)
    s.update(K=30, move=2, seed=5, kappa=1.0, mala_step=0.05)
    rng = np.random.default_rng(9)
    target = rng.uniform(0.25, 0.75, (2, 2, 3))
    A = rng.uniform(40.0, 120.0, (2, 6))

    def evaluate(u, J):
        d = (u - target[None]).reshape(u.shape[0], 2, 6)
        return 0.5 * (A[None] * d * d).sum(-1), np.ones((u.shape[0], 2), bool)

    def grad(u, J):
        d = (u - target[None]).reshape(u.shape[0], 2, 6)
        return (A[None] * d).reshape(u.shape)

    res = smc.run_smc(s, evaluate, 256, 30, 2, 2, grad=grad)
    assert np.abs(res["u"][res["best"]] - target).max() < 0.06
    assert 0.0 < np.mean(res["acc_rate"]) < 1.0
