"""Sequential Monte Carlo optimiser of one MPC update, plus the kernel-level
steps it is made of (initialisation, weighting, resampling, moves, final
selection).

Test infrastructure (CPU oracle); never part of the product path.

Paper passages followed:
  * Alg. 1 (Sequential Monte Carlo): initialise controls uniformly; repeat
    {sample disturbances, simulate, zero the weight of constraint violators,
    scale weights by the objective}; resample; perturb with Gaussian white
    noise; finally pick one particle;
  * Sec. "Particles": controls are initialised from a uniform distribution
    between each control's bounds; weights are kept per aircraft;
  * Sec. "Weight Scaling": the weight of aircraft i in particle l is the
    product of its objective values over the inner loop, 0 after any
    violation;
  * Sec. "Particle Resampling and Perturbation": aircraft are resampled
    independently of each other (Kitagawa-type, i.e. systematic resampling);
  * Sec. "Final Sample Selection": the particle maximising the product of its
    aircraft weights is returned; a particle with a violating aircraft cannot
    be chosen;
  * Sec. "Simulation Setup": SampleSchedule(J) = floor(3 + 5 exp(0.05 J)).

Build-specific readings (listed in the design notes): the inner loop draws M
wind samples per iteration and the growing SampleSchedule(J) becomes the
tempering exponent beta_J = kappa * SampleSchedule(J) of
log W = -beta_J * mean_m(cost) (a product of S(J) objective values is
exp(S(J) * mean log J)); with the paper's literal weighting (weighting 1)
iteration J makes S(J) + 1 passes, pass j under wind sample j, and
log W = sum_j log(1 - cost_j); resampling quantises the normalised weights to
integers so that its FP64 prefix sum is exact; an all-zero weight row keeps
its particles (identity ancestors); the random-walk move is a Metropolis step
on the joint particle with the product of aircraft weights as target.
"""
from __future__ import annotations

import bisect
import math

import numpy as np

from . import philox
from . import rollout as _rollout
from . import wind as _wind


# --- schedule and weights ----------------------------------------------------

def sample_schedule(J: int) -> int:
    """floor(3 + 5 e^{0.05 J}) (Sec. "Simulation Setup")."""
    return int(math.floor(3.0 + 5.0 * math.exp(0.05 * J)))


def beta(scen, J: int) -> float:
    return float(scen["kappa"]) * sample_schedule(J)


def init_particles(scen, mpc_step=None, L=None):
    """u[l, i, s, c] ~ U(0, 1), element e = ((l N + i) S + s) 3 + c."""
    L = scen["L"] if L is None else L
    N, S = scen["N"], scen["S"]
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    e = np.arange(L * N * S * 3, dtype=np.int64)
    u = philox.uniforms(scen["seed"], step, 0, philox.INIT, e,
                        scen.get("scenario_id", 0))
    return u.reshape(L, N, S, 3)


def warm_start_particles(scen, u_prev, mpc_step=None):
    """Initial population of a warm-started update (Sec. "Model Predictive
    Control", "Rolling Window": the window moves by the applied part, the
    first control segment).  Particle l's segment s is the previous update's
    final particle l's segment s + 1; the last segment, past the previous
    horizon, is drawn U(0, 1) as a fresh initialisation draws that element."""
    u_prev = np.asarray(u_prev, dtype=np.float64)
    L, N, S = u_prev.shape[0], scen["N"], scen["S"]
    u = np.empty_like(u_prev)
    u[:, :, :S - 1] = u_prev[:, :, 1:]
    u[:, :, S - 1] = init_particles(scen, mpc_step, L)[:, :, S - 1]
    return u


def expected_cost(cost, feas):
    """c_hat[l, i] = (1/M) sum_m cost[l, m, i] (exactly rounded sum),
    feasible[l, i] = all_m feas[l, m, i]."""
    L, M, N = cost.shape
    chat = np.empty((L, N))
    for l in range(L):
        for i in range(N):
            chat[l, i] = math.fsum(cost[l, :, i]) / M
    return chat, feas.all(axis=1)


def log_weights(chat, feasible, b):
    """log W = -beta * c_hat, or -inf for a violating aircraft."""
    return np.where(feasible, -b * chat, -np.inf)


def product_weighting(scen) -> bool:
    """The paper's literal weighting (Alg. 1 inner loop, Sec. "Weight
    Scaling") in place of the tempered mean."""
    return int(scen.get("weighting", 0)) == 1


def inner_samples(J: int) -> int:
    """Inner-loop passes of iteration J: j = 0 .. SampleSchedule(J)."""
    return sample_schedule(J) + 1


def product_log_weights(cost, feas):
    """Sec. "Weight Scaling": from W = 1/L every pass j multiplies the weight
    by the objective value J_T = 1 - cost (costs are 1 - J here), and a
    violation in any pass zeroes it: log W = sum_j log(1 - cost_j) up to the
    common log(1/L), or -inf.  cost, feas: [L, n, N] over the n passes."""
    L, n, N = cost.shape
    out = np.empty((L, N))
    for l in range(L):
        for i in range(N):
            if not feas[l, :, i].all():
                out[l, i] = -np.inf
                continue
            terms = [math.log1p(-c) if c < 1.0 else -math.inf for c in cost[l, :, i]]
            out[l, i] = -math.inf if -math.inf in terms else math.fsum(terms)
    return out


# --- resampling --------------------------------------------------------------

def quant_bits(L: int) -> int:
    """Kq = 52 - ceil(log2 L): L integers below 2^Kq sum to below 2^52."""
    return 52 - int(math.ceil(math.log2(L))) if L > 1 else 52


def quantised_weights(logw_row):
    """q_l = floor(exp(logw_l - max logw) * 2^Kq) as exact integers."""
    L = len(logw_row)
    mx = np.max(logw_row)
    w = np.exp(logw_row - mx)
    return [int(math.floor(wl * 2.0 ** quant_bits(L))) for wl in w]


def systematic_ancestors(q, U: int):
    """a_k = min{l : C_l L 2^32 > (k 2^32 + U) Q}, k = 0..L-1, with
    C_l = q_0 + ... + q_l and Q = C_{L-1}: systematic resampling with the
    single offset U / 2^32, evaluated in exact integer arithmetic."""
    L = len(q)
    C = []
    run = 0
    for ql in q:
        run += ql
        C.append(run)
    Q = C[-1]
    if Q == 0:
        return np.arange(L, dtype=np.int64)
    keys = [c * L * (1 << 32) for c in C]
    return np.array([bisect.bisect_right(keys, (k * (1 << 32) + U) * Q)
                     for k in range(L)], dtype=np.int64)


def resample_row(logw_row, U: int):
    """Ancestors of one aircraft row (identity if every weight is zero)."""
    L = len(logw_row)
    if not np.any(np.isfinite(logw_row)):
        return np.arange(L, dtype=np.int64)
    return systematic_ancestors(quantised_weights(logw_row), int(U))


def resample_offsets(scen, J, N, mpc_step=None):
    """U_i = first Philox word of (RESAMPLE, element i)."""
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    w = philox.words(scen["seed"], step, J, philox.RESAMPLE,
                     np.arange(N, dtype=np.int64), scen.get("scenario_id", 0))
    return [int(x) for x in w[0]]


def resample(logw, Us):
    """ancestors[i, k] for every aircraft row i (rows independent)."""
    L, N = logw.shape
    return np.stack([resample_row(logw[:, i], Us[i]) for i in range(N)])


def gather(u, anc):
    """u_new[k, i] = u[anc[i, k], i]."""
    L, N = u.shape[:2]
    out = np.empty_like(u)
    for i in range(N):
        out[:, i] = u[anc[i], i]
    return out


# --- moves -------------------------------------------------------------------

def move_normals(scen, J, shape, purpose=philox.MOVE, mpc_step=None):
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    n = int(np.prod(shape))
    xi = philox.normals(scen["seed"], step, J, purpose,
                        np.arange(n, dtype=np.int64), scen.get("scenario_id", 0))
    return xi.reshape(shape)


def jitter(scen, u, J, mpc_step=None):
    """Gaussian white-noise perturbation, clamped to the control box."""
    xi = move_normals(scen, J, u.shape, mpc_step=mpc_step)
    return np.clip(u + scen["sigma_move"] * xi, 0.0, 1.0)


def reflect(u):
    """Reflect into [0, 1] (symmetric, so the proposal stays symmetric)."""
    r = np.mod(u, 2.0)
    return np.where(r > 1.0, 2.0 - r, r)


def rw_propose(scen, u, J, mpc_step=None):
    xi = move_normals(scen, J, u.shape, mpc_step=mpc_step)
    return reflect(u + scen["sigma_move"] * xi)


def mh_accept(scen, J, logw, logw_prop, mpc_step=None, log_q_ratio=None):
    """Accept per particle with the joint target prod_i W_i:
    reject if the proposal violates; accept if the current state violates;
    otherwise accept iff log U < sum_i logw' - sum_i logw (+ log q ratio)."""
    L, N = logw.shape
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    U = philox.uniforms(scen["seed"], step, J, philox.ACCEPT,
                        np.arange(L, dtype=np.int64), scen.get("scenario_id", 0))
    acc = np.zeros(L, dtype=bool)
    for l in range(L):
        s_new = 0.0
        s_old = 0.0
        for i in range(N):
            s_new += logw_prop[l, i]
            s_old += logw[l, i]
        if s_new == -np.inf:
            acc[l] = False
        elif s_old == -np.inf:
            acc[l] = True
        else:
            d = s_new - s_old
            if log_q_ratio is not None:
                d += log_q_ratio[l]
            acc[l] = math.log(U[l]) < d
    return acc


# --- final selection ---------------------------------------------------------

def select_best(logw, chat, b):
    """Particle with the largest product of aircraft weights (sum of log
    weights), lowest index on ties.  If every particle has a violating
    aircraft: fewest violating aircraft first, then the largest sum of
    -beta * c_hat.  Returns (l*, infeasible flag)."""
    L, N = logw.shape
    best = None
    best_key = None
    for l in range(L):
        nbad = 0
        s = 0.0
        for i in range(N):
            if logw[l, i] == -np.inf:
                nbad += 1
            s += -b * chat[l, i]
        key = (-nbad, s)
        if best_key is None or key > best_key:
            best_key, best = key, l
    return best, best_key[0] < 0


# --- one MPC update ----------------------------------------------------------

def mala_propose(scen, u, g, J, mpc_step=None):
    """Langevin proposal in logit coordinates (MALA stream):
    u' = logistic(logit(u) + drift + eps xi), drift from `grad.mala_drift`."""
    from .grad import logistic, logit, mala_drift
    eps = scen["mala_step"]
    xi = move_normals(scen, J, u.shape, purpose=philox.MALA, mpc_step=mpc_step)
    return logistic(logit(u) + mala_drift(u, g, eps) + eps * xi)


def mala_log_ratio(scen, u, up, g, gp):
    """Per particle: whether the proposal u' lies inside the open box, and
    log q(theta | theta') - log q(theta' | theta) + log J(u') - log J(u) of
    the Langevin move in logit coordinates (J the Jacobian of the logit map;
    0 for a proposal on a face)."""
    from .grad import log_jacobian, mala_log_q
    eps = scen["mala_step"]
    L = u.shape[0]
    inside = np.all(((up > 0.0) & (up < 1.0)).reshape(L, -1), axis=1)
    up_safe = np.where(inside[:, None, None, None], up, u)
    lq = (mala_log_q(u, up_safe, gp, eps) - mala_log_q(up_safe, u, g, eps)
          + log_jacobian(up_safe) - log_jacobian(u))
    return inside, np.where(inside, lq, 0.0)


def mh_move(scen, u, chat, logw, J, b, evaluate, grad=None, mpc_step=None):
    """One Metropolis move of every particle on the joint target
    prod_i W_i = exp(-b sum_i c_hat_i) (zero if an aircraft violates) under
    the fields of iteration J: the random walk (move 1, reflected proposal,
    symmetric) or the Langevin proposal in logit coordinates (move 2, drift
    from g = -b grad; the ratio adds the proposal densities
    q(theta | theta') / q(theta' | theta) and the Jacobians
    prod u'(1 - u') / prod u(1 - u) of the logit map).  A Langevin proposal
    that rounds onto a face of the box (u' = 0 or 1, logit coordinate beyond
    about 37) is rejected: the carried target vanishes there.  Returns the
    moved particles, their c_hat and log-weights, the acceptance flags and
    the proposal's intermediates."""
    L = u.shape[0]
    if scen["move"] == 1:
        up = rw_propose(scen, u, J, mpc_step)
        ev = evaluate(up, J)
        chat_p, feas_p = ev[0], ev[1]
        logw_p = ev[2] if len(ev) > 2 else log_weights(chat_p, feas_p, b)
        acc = mh_accept(scen, J, logw, logw_p, mpc_step)
        extra = dict(u_prop=up)
    else:
        g = -b * grad(u, J)
        up = mala_propose(scen, u, g, J, mpc_step)
        chat_p, feas_p = evaluate(up, J)[:2]
        logw_p = log_weights(chat_p, feas_p, b)
        gp = -b * grad(up, J)
        inside, lq = mala_log_ratio(scen, u, up, g, gp)
        logw_p_eff = np.where(inside[:, None], logw_p, -np.inf)
        acc = mh_accept(scen, J, logw, logw_p_eff, mpc_step, log_q_ratio=lq)
        extra = dict(u_prop=up, g=g, g_prop=gp)
    u = np.where(acc[:, None, None, None], up, u)
    chat = np.where(acc[:, None], chat_p, chat)
    logw = np.where(acc[:, None], logw_p, logw)
    return u, chat, logw, acc, extra


def run_smc(scen, evaluate, L, K, N, S, mpc_step=None, trace=None,
            u_init=None, grad=None):
    """Generic SMC optimiser (Alg. 1 with the readings above).

    ``evaluate(u, J)`` -> (c_hat [L, N], feasible [L, N]) or (c_hat,
    feasible, log W) when it weights by itself; ``grad(u, J)`` ->
    d/du sum_i c_hat_i of the differentiable (fuel + time) part, needed by the
    Langevin move.  Returns dict with the final particles, c_hat,
    log-weights, the selected index and status."""
    move = scen["move"]
    u = init_particles(scen, mpc_step, L) if u_init is None else u_init.copy()
    acc_rate = []
    for J in range(K):
        b = beta(scen, J)
        ev = evaluate(u, J)
        chat, feas = ev[0], ev[1]
        logw = ev[2] if len(ev) > 2 else log_weights(chat, feas, b)
        if trace is not None:
            trace.append(dict(J=J, u=u.copy(), chat=chat.copy(), logw=logw.copy()))
        if move in (1, 2):
            u, chat, logw, acc, extra = mh_move(scen, u, chat, logw, J, b, evaluate,
                                                grad, mpc_step)
            acc_rate.append(float(acc.mean()))
            if trace is not None:
                trace[-1].update(acc=acc, logw_after=logw.copy(), **extra)
        if J == K - 1:
            break
        anc = resample(logw, resample_offsets(scen, J, N, mpc_step))
        if trace is not None:
            trace[-1]["anc"] = anc
        u = gather(u, anc)
        if move == 0:
            u = jitter(scen, u, J, mpc_step)
    b = beta(scen, K - 1)
    lstar, infeasible = select_best(logw, chat, b)
    return dict(u=u, chat=chat, logw=logw, best=lstar, infeasible=infeasible,
                acc_rate=acc_rate)


def physical(scen, u_norm):
    lo, hi = scen["ctrl_lo"], scen["ctrl_hi"]
    return lo + u_norm * (hi - lo)


def smc_mpc_step(scen, states=None, k_active=None, horizon=None, mpc_step=None,
                 trace=None, u_prev=None):
    """One MPC update: returns the optimised controls [N, S, 3] (physical),
    the expected cost (total, per aircraft) of the chosen particle and the
    infeasible flag.  With the scenario's warm start on and the previous
    update's final population u_prev [L, N, S, 3], the update starts from
    warm_start_particles instead of a fresh draw."""
    N, S, L, K = scen["N"], scen["S"], scen["L"], scen["K"]
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    Lfac = _wind.factor(scen)

    fields = {}

    def field(J):
        if J not in fields:
            fields.clear()
            fields[J] = _wind.sample_field(scen, J, step, Lfac)
        return fields[J]

    def evaluate(u, J):
        if product_weighting(scen):
            # pass j of the inner loop draws sample j of the iteration's fields
            r = _rollout.rollout(scen, u, field(J)[:inner_samples(J)], states, k_active, horizon)
            chat, feas = expected_cost(r["cost"], r["feas"])
            return chat, feas, product_log_weights(r["cost"], r["feas"])
        r = _rollout.rollout(scen, u, field(J), states, k_active, horizon)
        return expected_cost(r["cost"], r["feas"])

    def grad(u, J):
        from .grad import grad_fuel_time
        return grad_fuel_time(scen, u, field(J), states, k_active, horizon)[1]

    u_init = None
    if scen.get("warm_start", 0) and u_prev is not None:
        u_init = warm_start_particles(scen, u_prev, step)
    res = run_smc(scen, evaluate, L, K, N, S, step, trace, u_init=u_init, grad=grad)
    l = res["best"]
    per = res["chat"][l]
    total = 0.0
    for i in range(N):
        total += per[i]
    return dict(controls=physical(scen, res["u"][l]), u_best=res["u"][l].copy(),
                best=l, cost=total, cost_per=per.copy(),
                infeasible=res["infeasible"], result=res)


def eval_cost(scen, particles, J, states=None, k_active=None, horizon=None,
              mpc_step=None):
    """Expected cost and feasibility of given normalised particles
    [P, N, S, 3] under the wind fields of iteration J."""
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    W = _wind.sample_field(scen, J, step)
    r = _rollout.rollout(scen, particles, W, states, k_active, horizon)
    return expected_cost(r["cost"], r["feas"])
