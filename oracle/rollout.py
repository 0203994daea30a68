"""Trajectory rollout of every (particle, wind sample, aircraft): dynamics,
unary constraints, landing test, per-step cost terms and pairwise separation.

Test infrastructure (CPU oracle); never part of the product path.

Plain FP64 NumPy over arrays of shape (L, M, N) = (particles, wind samples,
aircraft); the time loop is a Python loop in the paper's order.

Paper passages followed:
  * Sec. "Trajectory Planning and Disturbance Realisations", eq. (hor):
    explicit Euler update of (x, y, z, v, chi, m) with the wind added to
    x and y;
  * the inverse relations of Sec. "Fuel Estimate 1" (eqs. for eta, gamma and
    T) and "Fuel Estimate 2" (bank from heading change) map the library's
    per-segment kinematic controls (heading rate, airspeed, climb rate) onto
    the paper's thrust / climb angle / bank angle; the airspeed control is
    the speed reached at the end of its segment, approached linearly
    (v_{k+1} = v_k + (v_c - v_k) / (k_end - k));
  * Sec. "Constraint Handling": unary envelope and minimum-mass constraints;
    eq. (avoidance): a pair is safe at a step if its horizontal distance is at
    least 2 P_r or its vertical distance at least 2 P_h; a violation zeroes
    both aircraft;
  * eq. (TO_init): the landing sector test for arrivals; Sec. "Rolling
    Window": a landed arrival leaves the problem and scores the best cost for
    the remaining steps; an aircraft is optimised from its activation step;
  * Sec. "Particle Costing": every objective element is negated and
    normalised to [0, 1] by its supremum and infimum; departures use bearing,
    fuel, altitude and speed, arrivals flow-field heading, nominal glide and
    fuel; Sec. "Noise Pollution Reduction": the altitude-weighted population
    noise term.

The paper's own control parametrisation (control_model 1, Sec.
"Trajectory Planning and Disturbance Realisations", eq. (hor) and Sec.
"Particles"): every step k has its own controls, thrust T (a fraction of
T_max), flight-path angle gamma and bank angle phi; v' = v + dt ((T - D)/m -
g sin gamma), chi' = chi + dt L sin(phi) / (m v) with the lift of the
coordinated turn L = m g cos(gamma) / cos(phi), z' = z + dt v sin(gamma),
m' = m - dt eta(v) T.

Build-specific readings (all listed in the design notes): costs are
minimised, c = 1 - J per element, so the best cost is 0; a time-to-go term is
added; the flow field is chi_hat = pi + 2 atan2(y, x) with remaining arc
length s_arc = r |theta| / sin|theta|; the nominal glide angle is
atan2(z, s_arc); fuel burn is clamped at zero thrust; the sums over the
horizon are divided by H once.
"""
from __future__ import annotations

import math

import numpy as np

from . import wind as _wind

G0 = 9.80665                      # gravity [m/s^2]
RHO0, T0, LAPSE, R_AIR = 1.225, 288.15, 0.0065, 287.05287
ISA_EXP = G0 / (R_AIR * LAPSE) - 1.0


def isa_density(z):
    """ISA troposphere density; altitude clamped to [0, 11 km]."""
    zc = np.clip(z, 0.0, 11_000.0)
    return RHO0 * (1.0 - LAPSE * zc / T0) ** ISA_EXP


def wrap(a):
    """Angle wrapped to [-pi, pi)."""
    return a - 2.0 * math.pi * np.floor((a + math.pi) / (2.0 * math.pi))


def arc_ratio(theta_abs):
    """|theta| / sin|theta| (length of the flow-field arc over the radius)."""
    safe = np.maximum(np.sin(theta_abs), 1e-6)
    return np.where(theta_abs > 1e-4, theta_abs / safe,
                    1.0 + theta_abs * theta_abs / 6.0)


def bilinear(grid2d, box, x, y):
    """Bilinear interpolation of a [ny, nx] grid spanning the box, clamped."""
    ny, nx = grid2d.shape
    wx, wy = float(box[0]), float(box[1])
    fx = np.clip((x + wx / 2) / (wx / (nx - 1)), 0.0, nx - 1)
    fy = np.clip((y + wy / 2) / (wy / (ny - 1)), 0.0, ny - 1)
    ix = np.minimum(np.floor(fx).astype(np.int64), nx - 2)
    iy = np.minimum(np.floor(fy).astype(np.int64), ny - 2)
    tx, ty = fx - ix, fy - iy
    g = grid2d.astype(np.float64)
    return ((1 - tx) * (1 - ty) * g[iy, ix] + tx * (1 - ty) * g[iy, ix + 1]
            + (1 - tx) * ty * g[iy + 1, ix] + tx * ty * g[iy + 1, ix + 1])


def landing_conditions(scen, x, y, z, v, chi):
    """The five landing-sector conditions of eq. (TO_init) as a list of
    (lhs, rhs) pairs, each satisfied when lhs <= rhs."""
    p_run, p_beta, p_chi, p_vs, _ = scen["landing"]
    r = np.hypot(x, y)
    theta = np.arctan2(y, x)
    s_arc = r * arc_ratio(np.abs(theta))
    beta = np.arctan2(z, s_arc)
    return [(r, p_run), (beta, p_beta), (np.abs(theta), p_chi),
            (np.abs(wrap(chi - math.pi)), p_chi), (v, p_vs)]


def time_element(scen, x, y, v):
    """Time-to-go element min(t_go / t_norm, 1): arrivals fly the remaining
    flow-field arc, departures the remaining distance to the exit radius."""
    kind = scen["kind"]
    vv = np.maximum(v, scen["env"][2])
    r = np.hypot(x, y)
    s_arc = r * arc_ratio(np.abs(np.arctan2(y, x)))
    dtma = scen["targets"][:, 3]
    t_arr = np.minimum(s_arc / vv / scen["time_norm"], 1.0)
    t_dep = np.minimum(np.maximum(dtma - r, 0.0) / vv / scen["time_norm"], 1.0)
    return np.where(kind == 0, t_arr, t_dep)


def climb_rate_bound(scen):
    """Largest climb or descent rate the controls allow [m/s]: the climb-rate
    bound of the kinematic controls, or v_max sin(gamma_bound) for the
    paper's flight-path-angle control."""
    lo, hi = scen["ctrl_lo"], scen["ctrl_hi"]
    if scen.get("control_model", 0) == 1:
        return scen["env"][3] * math.sin(max(abs(lo[1]), abs(hi[1])))
    return max(abs(lo[2]), abs(hi[2]))


def step_cost(scen, j, x, y, z, v, chi, z_act):
    """Per-step cost (0 best, 1 worst) at a new state, for every aircraft.

    ``j`` = steps since activation (>= 1), ``z_act`` = altitude at
    activation.  Arrays broadcast over (L, M, N)."""
    kind = scen["kind"]
    w = scen["cost_w"]
    a_time, a_noise = w[7], w[8]
    mix = 1.0 - a_time - a_noise
    vmin, vmax = scen["env"][2], scen["env"][3]
    beta_f = scen["landing"][4]
    theta_F, Zt, vD, dtma = (scen["targets"][:, c] for c in range(4))
    zdot_max = climb_rate_bound(scen)
    dt = scen["dt"]

    theta = np.arctan2(y, x)
    r = np.hypot(x, y)
    vv = np.maximum(v, vmin)
    # arrival elements: heading off the flow field, nominal glide angle
    chi_hat = math.pi + 2.0 * theta
    hdg = np.abs(wrap(chi - chi_hat)) / math.pi
    s_arc = r * arc_ratio(np.abs(theta))
    beta = np.arctan2(z, s_arc)
    glide = np.abs(beta - beta_f) / (math.pi / 2.0)
    t_arr = np.minimum(s_arc / vv / scen["time_norm"], 1.0)
    # departure elements: bearing, altitude (reachable band), speed
    brg = np.abs(wrap(theta - theta_F)) / math.pi
    d0 = np.abs(Zt - z_act)
    span = zdot_max * j * dt
    sup = d0 + span
    inf = np.maximum(d0 - span, 0.0)
    alt = np.clip((np.abs(Zt - z) - inf) / (sup - inf), 0.0, 1.0)
    spd = np.abs(v - vD) / np.maximum(vmax - vD, vD - vmin)
    t_dep = np.minimum(np.maximum(dtma - r, 0.0) / vv / scen["time_norm"], 1.0)
    if a_noise != 0.0 and scen.get("popdense") is not None:
        A_c = scen["noise_alt"]
        noise = (np.maximum(1.0 - (z / A_c) ** 2, 0.0)
                 * bilinear(scen["popdense"], scen["box"], x, y))
    else:
        noise = 0.0
    c_arr = mix * (w[0] * hdg + w[1] * glide) + a_time * t_arr + a_noise * noise
    c_dep = (mix * (w[3] * brg + w[5] * alt + w[6] * spd) + a_time * t_dep
             + a_noise * noise)
    return np.where(kind == 0, c_arr, c_dep)


def rollout(scen, u_norm, W, states=None, k_active=None, horizon=None,
            with_margins=False, record=False):
    """Roll out particles ``u_norm`` [L, N, S, 3] (normalised controls in
    [0, 1]) under wind fields ``W`` [M, G, 2], or [H, M, G, 2] with one
    field per step (the paper's time-correlated model).

    Returns dict with cost [L, M, N], ft_cost [L, M, N] (its fuel + time part),
    feas [L, M, N] (bool), steps (number of
    simulated aircraft-steps), pair_tests (separation tests with both aircraft
    present), and, if asked, margin [L, M, N]: the smallest
    relative distance of any discrete decision (unary check, landing test,
    separation test) to its threshold; if ``record``, track [H+1, L, M, N, 6]
    (state after each step, frozen once an aircraft is absent) and present
    [H, L, M, N] (aircraft simulated at step k)."""
    states = scen["states"] if states is None else states
    k_active = scen["k_active"] if k_active is None else k_active
    H = scen["H"] if horizon is None else int(horizon)
    N, S, dt = scen["N"], scen["S"], scen["dt"]
    L, M = u_norm.shape[0], (W.shape[1] if W.ndim == 4 else W.shape[0])
    ac = scen["aircraft"]
    Sw, cd0, cd2, cf1, cf2, tmax, m_empty, phi_max, gamma_max = ac.T
    zmin, zmax, vmin, vmax = scen["env"]
    lo, hi = scen["ctrl_lo"], scen["ctrl_hi"]
    u = lo + u_norm * (hi - lo)                   # physical controls
    is_arr = scen["kind"] == 0
    kact = np.asarray(k_active, dtype=np.int64)
    active = (kact >= 0) & (kact < H)
    n_steps = np.where(active, H - kact, 0)
    shape = (L, M, N)

    x, y, z, v, chi, mass = (np.broadcast_to(states[:, c], shape).astype(np.float64)
                             for c in range(6))
    z_act = z.copy()
    m_act = mass.copy()
    feas = np.ones(shape, dtype=bool)
    done = np.zeros(shape, dtype=bool)
    acc = np.zeros(shape)
    acc_t = np.zeros(shape)
    margin = np.full(shape, np.inf)
    m_idx = np.arange(M)[None, :, None]
    steps = 0
    pair_tests = 0
    p_sep_h2, p_sep_v = scen["sep_h"] ** 2, scen["sep_v"]
    track = [np.stack([x, y, z, v, chi, mass], axis=-1)] if record else None
    pres_log = [] if record else None

    paper_controls = scen.get("control_model", 0) == 1
    if paper_controls and S < H:
        raise ValueError("the per-step controls need a control set for every step (S >= H)")
    for k in range(H):
        present = active & (k >= kact) & ~done
        steps += int(present.sum())
        Wk = W[k] if W.ndim == 4 else W           # per-step fields (paper's model)
        wxy = _wind.trilinear(Wk, m_idx, scen["box"], scen["grid"], x, y, z)
        rho = isa_density(z)
        qd = 0.5 * rho * v * v
        eta = cf1 * (1.0 + v / cf2)
        if paper_controls:
            # thrust, flight-path angle and bank of step k (eq. hor)
            T = np.broadcast_to(u[:, None, :, k, 0] * tmax, shape)
            gamma = np.broadcast_to(u[:, None, :, k, 1], shape)
            phi = np.broadcast_to(u[:, None, :, k, 2], shape)
            lift = mass * G0 * np.cos(gamma) / np.cos(phi)   # coordinated turn
            CL = lift / (qd * Sw)
            CD = cd0 + cd2 * CL * CL
            D = qd * Sw * CD
            vn = v + dt * ((T - D) / mass - G0 * np.sin(gamma))
            chin = chi + dt * lift * np.sin(phi) / (mass * v)
            fuel = dt * eta * T
        else:
            s = (k * S) // H
            k_end = ((s + 1) * H + S - 1) // S    # first step of segment s+1
            chidot = u[:, None, :, s, 0]
            vc = u[:, None, :, s, 1]
            zdot = u[:, None, :, s, 2]
            gamma = np.arcsin(zdot / v)           # climb angle from climb rate
            phi = np.arctan(v * chidot / G0)      # bank for the heading rate
            CL = mass * G0 / (qd * Sw * np.cos(phi))  # lift balances weight in turn
            CD = cd0 + cd2 * CL * CL
            D = qd * Sw * CD
            vn = v + (vc - v) / (k_end - k)       # ramp to vc by segment end
            T = mass * (vn - v) / dt + D + mass * G0 * np.sin(gamma)
            fuel = dt * eta * np.maximum(T, 0.0)
            chin = chi + dt * chidot

        xn = x + dt * (v * np.cos(chi) * np.cos(gamma) + wxy[..., 0])
        yn = y + dt * (v * np.sin(chi) * np.cos(gamma) + wxy[..., 1])
        zn = z + dt * v * np.sin(gamma)
        mn = mass - fuel

        viol = ((T > tmax) | (np.abs(phi) >= phi_max) | (np.abs(gamma) > gamma_max)
                | (zn < zmin) | (zn > zmax) | (vn < vmin) | (vn > vmax)
                | (mn < m_empty))
        if with_margins:   # only decisions that can still change feasibility
            relevant = present & feas
            mg = np.minimum.reduce([
                np.abs(T - tmax) / tmax,
                np.abs(np.abs(phi) - phi_max) / phi_max,
                np.abs(np.abs(gamma) - gamma_max) / gamma_max,
                np.abs(zn - zmin) / zmax, np.abs(zn - zmax) / zmax,
                np.abs(vn - vmin) / vmax, np.abs(vn - vmax) / vmax,
                np.abs(mn - m_empty) / m_empty])
            margin = np.where(relevant, np.minimum(margin, mg), margin)
        feas &= ~(present & viol)

        x = np.where(present, xn, x)
        y = np.where(present, yn, y)
        z = np.where(present, zn, z)
        v = np.where(present, vn, v)
        chi = np.where(present, chin, chi)
        mass = np.where(present, mn, mass)

        conds = landing_conditions(scen, x, y, z, v, chi)
        ok = [lhs <= rhs for lhs, rhs in conds]
        landed = present & is_arr & np.logical_and.reduce(ok)
        if with_margins:
            for c_idx, (lhs, rhs) in enumerate(conds):
                others = np.logical_and.reduce([ok[o] for o in range(5) if o != c_idx])
                mg = np.abs(lhs - rhs) / abs(rhs)
                upd = present & is_arr & others
                margin = np.where(upd, np.minimum(margin, mg), margin)

        if record:
            track.append(np.stack([x, y, z, v, chi, mass], axis=-1))
            pres_log.append(present.copy())
        j = np.maximum(k + 1 - kact, 1)           # steps since activation
        c = step_cost(scen, j, x, y, z, v, chi, z_act)
        acc += np.where(present & ~landed, c, 0.0)
        acc_t += np.where(present & ~landed, time_element(scen, x, y, v), 0.0)
        done |= landed

        # pairwise separation among aircraft that have a state at k+1
        for i in range(N):
            for jj in range(i + 1, N):
                both = present[..., i] & present[..., jj]
                pair_tests += int(both.sum())
                dh2 = (x[..., i] - x[..., jj]) ** 2 + (y[..., i] - y[..., jj]) ** 2
                dz = np.abs(z[..., i] - z[..., jj])
                A = dh2 < p_sep_h2
                B = dz < p_sep_v
                bad = both & A & B
                if with_margins:
                    mg = np.minimum(np.where(B, np.abs(dh2 / p_sep_h2 - 1.0), np.inf),
                                    np.where(A, np.abs(dz / p_sep_v - 1.0), np.inf))
                    mg = np.where(both & (feas[..., i] | feas[..., jj]), mg, np.inf)
                    margin[..., i] = np.minimum(margin[..., i], mg)
                    margin[..., jj] = np.minimum(margin[..., jj], mg)
                feas[..., i] &= ~bad
                feas[..., jj] &= ~bad

    w = scen["cost_w"]
    mix = 1.0 - w[7] - w[8]
    a_fuel = np.where(is_arr, w[2], w[4])
    denom = dt * np.maximum(n_steps, 1) * tmax * (cf1 * (1.0 + vmax / cf2))
    fuel_term = (m_act - mass) / denom
    cost = np.where(active, mix * a_fuel * fuel_term + acc / np.maximum(n_steps, 1),
                    0.0)
    # the differentiable part used by gradient-informed moves: fuel + time
    ft_cost = np.where(active, mix * a_fuel * fuel_term
                       + w[7] * acc_t / np.maximum(n_steps, 1), 0.0)
    out = dict(cost=cost, feas=feas, steps=steps, pair_tests=pair_tests, ft_cost=ft_cost,
               final=np.stack([x, y, z, v, chi, mass], axis=-1))
    if with_margins:
        out["margin"] = margin
    if record:
        out["track"] = np.stack(track)
        out["present"] = np.stack(pres_log)
    return out
