"""Receding-horizon loop around the SMC optimiser (test infrastructure only).

Sec. "Model Predictive Control": at each update the optimiser returns a
control sequence over the horizon H from the measured states; only its first
part is applied to the plant, whose disturbance (the wind) differs from the
optimiser's predictions.  Sec. "Rolling Window": the window of length H moves
with every completed update; an aircraft joins the problem at its
pre-determined step and is optimised only while active; an arrival leaves
the problem once it has landed.

Readings (the paper is silent): the applied part is the first control
segment, ceil(H / S) steps; the plant flies the plan with the rollout's
arithmetic through one wind sample, sample 0 of the fields the optimiser
would draw for an iteration word it never uses (``plant_iter``): one static
field, or under the paper's time-correlated model (Sec. "Wind Model") that
sample's field of each step; a departure
leaves the problem once it is outside its exit radius D_TMA; the plant's
states are exact (no observer).
"""
from __future__ import annotations

import math

import numpy as np

from . import rollout as _rollout
from . import smc as _smc
from . import wind as _wind


def applied_steps(scen, horizon=None) -> int:
    """Length of the first control segment: the steps applied per update."""
    H = scen["H"] if horizon is None else int(horizon)
    return int(math.ceil(H / scen["S"]))


def plant_step(scen, controls, states, k_active, n_steps, plant_iter, mpc_step,
               horizon=None, Lfac=None):
    """Advance the plant n_steps steps under the plan ``controls`` [N, S, 3]
    (physical).  Returns (states [N, 6], k_active [N], event [N]) after the
    steps: k_active shifts by n_steps (an aircraft that joined is now 0), an
    arrival that landed or a departure outside its exit radius leaves the
    problem (k_active -1); event is 1 landed, 2 left through the exit
    radius, 0 otherwise.  An aircraft that has not joined keeps its state."""
    H = scen["H"] if horizon is None else int(horizon)
    N = scen["N"]
    lo, hi = scen["ctrl_lo"], scen["ctrl_hi"]
    u = ((np.asarray(controls, dtype=np.float64) - lo) / (hi - lo))[None]
    W = _wind.sample_field(scen, plant_iter, mpc_step, Lfac)
    # sample 0: its static field, or its field of every step [H, 1, G, 2]
    W = W[:, :1] if W.ndim == 4 else W[:1]
    r = _rollout.rollout(scen, u, W, states, k_active, H, record=True)
    track, present = r["track"][:, 0, 0], r["present"][:, 0, 0]     # [H+1, N, 6], [H, N]
    is_arr = scen["kind"] == 0
    landed = np.zeros(N, dtype=bool)
    for k in range(n_steps):
        x, y, z, v, chi = (track[k + 1][:, c] for c in range(5))
        ok = np.logical_and.reduce([lhs <= rhs for lhs, rhs in
                                    _rollout.landing_conditions(scen, x, y, z, v, chi)])
        landed |= present[k] & is_arr & ok
    new_states = track[n_steps].copy()
    kact = np.asarray(k_active, dtype=np.int64)
    k_new = np.where(kact < 0, -1, np.maximum(kact - n_steps, 0))
    r_xy = np.hypot(new_states[:, 0], new_states[:, 1])
    joined = (kact >= 0) & (kact < n_steps)
    exited = joined & ~is_arr & (r_xy >= scen["targets"][:, 3])
    event = np.where(landed, 1, np.where(exited, 2, 0))
    k_new = np.where(event > 0, -1, k_new)
    return new_states, k_new.astype(np.int32), event.astype(np.int32)


def rolling_window(scen, n_updates, plant_iter=None, Lfac=None):
    """n_updates receding-horizon updates from the scenario's states: solve
    (Alg. 1), apply the first segment to the plant, shift the window (with
    the scenario's warm start on, each update after the first starts from
    the previous update's final population shifted by that segment).
    Returns a list of per-update dicts (controls, cost, states after the
    plant step, k_active, events)."""
    plant_iter = scen["K"] + 1 if plant_iter is None else plant_iter
    if Lfac is None:
        Lfac = _wind.factor(scen)
    states = np.array(scen["states"], dtype=np.float64)
    kact = np.array(scen["k_active"], dtype=np.int32)
    n = applied_steps(scen)
    out = []
    u_prev = None
    for t in range(n_updates):
        step = int(scen["mpc_step"]) + t
        res = _smc.smc_mpc_step(scen, states=states, k_active=kact, mpc_step=step,
                                u_prev=u_prev)
        u_prev = res["result"]["u"]
        states, kact, ev = plant_step(scen, res["controls"], states, kact, n, plant_iter,
                                      step, Lfac=Lfac)
        out.append(dict(controls=res["controls"], cost=res["cost"], states=states.copy(),
                        k_active=kact.copy(), event=ev))
    return out
