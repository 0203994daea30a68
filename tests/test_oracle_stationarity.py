"""Fixed-temperature stationarity of the oracle's Metropolis moves (Alg. 1
perturbation step, read as a Metropolis move on the joint target
prod_i W_i = exp(-beta sum_i c_hat_i)).

On the separable toy quadratic c = 1/2 (u - u*)^T A (u - u*) with diagonal A
and u* well inside the box, the target at a fixed beta is, up to mass beyond
the box faces that is below 1e-9 here, the Gaussian N(u*, (beta A)^-1).  A
move that is exact for that target must carry a population drawn away from
it (mean offset by several standard deviations) to a population whose mean is
u* and whose per-coordinate variance is 1 / (beta A), to within Monte Carlo
error.  The step is the oracle's own `smc.mh_move`; a fresh random stream per
step comes from the MPC-step counter word.  A reversed Langevin density ratio
(q(u' | u) / q(u | u') in place of q(u | u') / q(u' | u)) is planted in the
oracle and must fail the same check."""
import numpy as np
import pytest

from oracle import grad as og
from oracle import smc
from tests.oracle_helpers import mini

L_CHAINS = 4000
N, S = 1, 2                      # D = 6 coordinates


def _toy(near_face=False):
    rng = np.random.default_rng(11)
    if near_face:
        # 6 standard deviations from the face u = 0: mass beyond it < 1e-9
        target = rng.uniform(0.09, 0.11, (N, S, 3))
        A = rng.uniform(450.0, 550.0, (N, S, 3))
    else:
        target = rng.uniform(0.35, 0.65, (N, S, 3))
        A = rng.uniform(60.0, 140.0, (N, S, 3))
    return target, A


def _run(move, steps, eps=None, sigma=None, q_reversed=False, jac_dropped=False,
         near_face=False, monkeypatch=None):
    target, A = _toy(near_face)
    s = mini(N=N, S=S, L=L_CHAINS)
    s.update(move=move, seed=21, kappa=1.0,
             sigma_move=0.02 if sigma is None else sigma,
             mala_step=0.1 if eps is None else eps)
    J = 0
    b = smc.beta(s, J)           # 8: a fixed temperature for every step

    def evaluate(u, J_):
        d = u - target[None]
        return (0.5 * (A[None] * d * d).reshape(u.shape[0], N, -1).sum(-1),
                np.ones((u.shape[0], N), bool))

    def grad(u, J_):
        return A[None] * (u - target[None])

    if q_reversed:
        real = og.mala_log_q
        monkeypatch.setattr(og, "mala_log_q",
                            lambda u_to, u_from, g_from, e: -real(u_to, u_from, g_from, e))
    if jac_dropped:
        monkeypatch.setattr(og, "log_jacobian", lambda u: np.zeros(u.shape[0]))
    sd = 1.0 / np.sqrt(b * A)
    rng = np.random.default_rng(5)
    # start 3 standard deviations off the target mean, at the target's spread
    u = target[None] + 3.0 * sd[None] + sd[None] * rng.standard_normal((L_CHAINS, N, S, 3))
    chat, feas = evaluate(u, J)
    logw = smc.log_weights(chat, feas, b)
    acc = []
    for t in range(steps):
        u, chat, logw, a, _ = smc.mh_move(s, u, chat, logw, J, b, evaluate, grad,
                                          mpc_step=1000 + t)
        acc.append(a.mean())
    return u, target, sd, float(np.mean(acc))


def _stationarity_error(u, target, sd):
    """Largest |mean - u*| in units of the Monte Carlo standard error, and
    the largest |var / (1 / (beta A)) - 1| over the coordinates."""
    z = (u - target[None]) / sd[None]
    mean_z = z.mean(0)
    var_ratio = z.var(0)
    return float(np.abs(mean_z).max() * np.sqrt(L_CHAINS)), float(np.abs(var_ratio - 1).max())


# Monte Carlo bounds: the mean of 4000 independent chains has standard error
# sd / 63; the variance ratio has standard error sqrt(2 / 4000) = 0.022.
MEAN_SE_MAX = 5.0
VAR_REL_MAX = 0.10


@pytest.mark.parametrize("move,steps", [(1, 400), (2, 150)])
def test_move_leaves_gaussian_target_stationary(move, steps):
    u, target, sd, acc = _run(move, steps)
    mean_se, var_rel = _stationarity_error(u, target, sd)
    assert 0.05 < acc < 0.99, acc
    assert mean_se < MEAN_SE_MAX, mean_se
    assert var_rel < VAR_REL_MAX, var_rel


def test_langevin_move_is_stationary_near_a_face():
    u, target, sd, acc = _run(2, 150, near_face=True)
    mean_se, var_rel = _stationarity_error(u, target, sd)
    assert 0.05 < acc < 0.99, acc
    assert mean_se < MEAN_SE_MAX, mean_se
    assert var_rel < VAR_REL_MAX, var_rel


def test_dropped_jacobian_breaks_stationarity(monkeypatch):
    """Without the Jacobian of the logit map the chain targets
    exp(-beta c) / (u (1 - u)) instead: near the face u = 0 its mean moves
    towards the face by var * (1 - 2u) / (u (1 - u)), about 9 Monte Carlo
    standard errors here."""
    u, target, sd, acc = _run(2, 150, jac_dropped=True, near_face=True,
                              monkeypatch=monkeypatch)
    mean_se, var_rel = _stationarity_error(u, target, sd)
    assert mean_se >= MEAN_SE_MAX or var_rel >= VAR_REL_MAX, (mean_se, var_rel)


def test_langevin_drift_is_the_log_gradient_in_logit_coordinates():
    """(eps^2 / 2) d/dtheta [log pi(logistic(theta)) + log |du/dtheta|] by
    central differences equals the oracle's drift, for a target with a known
    gradient in u."""
    rng = np.random.default_rng(3)
    u = rng.uniform(0.02, 0.98, (4, 1, 2, 3))
    c = rng.normal(size=u.shape)

    def log_target_theta(t):
        uu = og.logistic(t)
        return np.sum(np.sin(3.0 * uu) * c) + np.sum(np.log(uu) + np.log1p(-uu))

    g = 3.0 * np.cos(3.0 * u) * c            # gradient in u of sum sin(3u) c
    eps, h = 0.2, 1e-6
    t = og.logit(u)
    fd = np.zeros_like(u)
    for idx in np.ndindex(u.shape):
        tp, tm = t.copy(), t.copy()
        tp[idx] += h
        tm[idx] -= h
        fd[idx] = (log_target_theta(tp) - log_target_theta(tm)) / (2 * h)
    assert np.allclose(og.mala_drift(u, g, eps), 0.5 * eps * eps * fd, rtol=1e-6, atol=1e-9)


def test_reversed_langevin_ratio_breaks_stationarity(monkeypatch):
    """The same check catches a Langevin acceptance with the density ratio
    reversed (the planted mistake lives in the oracle, on the CPU)."""
    u, target, sd, acc = _run(2, 150, q_reversed=True, monkeypatch=monkeypatch)
    mean_se, var_rel = _stationarity_error(u, target, sd)
    assert mean_se >= MEAN_SE_MAX or var_rel >= VAR_REL_MAX, (mean_se, var_rel)
