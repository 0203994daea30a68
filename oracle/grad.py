"""Reference gradient of the fuel + time part of the cost with respect to the
normalised controls, for the gradient-informed (MALA) move.

Test infrastructure (CPU oracle); never part of the product path.

The paper's optimiser is derivative-free; the gradient-informed move is a
build addition.  Only the proposal uses the gradient, and the Metropolis
acceptance is taken with the full target (every cost element and the
separation indicator), so the move keeps the SMC target.

`fuel_time_torch` transcribes the rollout of `oracle.rollout` for the fuel
element and the time-to-go element in PyTorch float64 on the CPU, so that
autograd gives the reference gradient.  Discrete events (landing, violation)
are taken as fixed by the forward pass: they carry no gradient.  Clamps,
max(T, 0) and min(t, 1) take the derivative of the active branch.  The
transcription is pinned by (i) equality of its value with the NumPy oracle's
`ft_cost` and (ii) central finite differences of that NumPy value (tests).
"""
from __future__ import annotations

import numpy as np

from . import rollout as _ro


def _trilinear_t(torch, W, m_idx, box, grid_n, x, y, z):
    wx, wy, zt = (float(b) for b in box)
    nx, ny, nz = (int(n) for n in grid_n)
    fx = torch.clamp((x + wx / 2) / (wx / (nx - 1)), 0.0, nx - 1)
    fy = torch.clamp((y + wy / 2) / (wy / (ny - 1)), 0.0, ny - 1)
    fz = torch.clamp(z / (zt / (nz - 1)), 0.0, nz - 1)
    ix = torch.clamp(torch.floor(fx.detach()).long(), max=nx - 2)
    iy = torch.clamp(torch.floor(fy.detach()).long(), max=ny - 2)
    iz = torch.clamp(torch.floor(fz.detach()).long(), max=nz - 2)
    tx, ty, tz = fx - ix, fy - iy, fz - iz
    out_x = torch.zeros_like(x)
    out_y = torch.zeros_like(x)
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                wgt = ((tx if a else 1 - tx) * (ty if b else 1 - ty) * (tz if c else 1 - tz))
                g = ((ix + a) * ny + (iy + b)) * nz + (iz + c)
                Wv = W[m_idx, g]
                out_x = out_x + wgt * Wv[..., 0]
                out_y = out_y + wgt * Wv[..., 1]
    return out_x, out_y


def fuel_time_torch(scen, u_norm, W, states=None, k_active=None, horizon=None):
    """Fuel + time cost [L, M, N] as a differentiable function of the
    normalised controls u_norm (torch float64 tensor [L, N, S, 3])."""
    import torch
    states = scen["states"] if states is None else states
    k_active = scen["k_active"] if k_active is None else k_active
    H = scen["H"] if horizon is None else int(horizon)
    N, S, dt = scen["N"], scen["S"], scen["dt"]
    L, M = u_norm.shape[0], W.shape[0]
    f64 = torch.float64
    T_ = lambda a: torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=f64)
    ac = T_(scen["aircraft"])
    Sw, cd0, cd2, cf1, cf2, tmax = (ac[:, c] for c in range(6))
    zmin, zmax, vmin, vmax = (float(e) for e in scen["env"])
    lo, hi = T_(scen["ctrl_lo"]), T_(scen["ctrl_hi"])
    u = lo + u_norm * (hi - lo)
    is_arr = torch.as_tensor(scen["kind"] == 0)
    kact = np.asarray(k_active, dtype=np.int64)
    active = torch.as_tensor((kact >= 0) & (kact < H))
    n_steps = torch.as_tensor(np.where((kact >= 0) & (kact < H), H - kact, 0))
    kact_t = torch.as_tensor(kact)
    Wt = T_(W)
    st = T_(states)
    shape = (L, M, N)
    x, y, z, v, chi, mass = (st[:, c].expand(shape).clone() for c in range(6))
    m_act = mass.clone()
    done = torch.zeros(shape, dtype=torch.bool)
    acc_t = torch.zeros(shape, dtype=f64)
    m_idx = torch.arange(M)[None, :, None].expand(shape)
    g0 = _ro.G0
    dtma = T_(scen["targets"][:, 3])
    for k in range(H):
        s = (k * S) // H
        k_end = ((s + 1) * H + S - 1) // S
        chidot = u[:, None, :, s, 0]
        vc = u[:, None, :, s, 1]
        zdot = u[:, None, :, s, 2]
        present = active & (k >= kact_t) & ~done
        wx, wy = _trilinear_t(torch, Wt, m_idx, scen["box"], scen["grid"], x, y, z)
        gamma = torch.asin(zdot / v)
        phi = torch.atan(v * chidot / g0)
        zc = torch.clamp(z, 0.0, 11_000.0)
        rho = _ro.RHO0 * (1.0 - _ro.LAPSE * zc / _ro.T0) ** _ro.ISA_EXP
        qd = 0.5 * rho * v * v
        CL = mass * g0 / (qd * Sw * torch.cos(phi))
        D = qd * Sw * (cd0 + cd2 * CL * CL)
        vn = v + (vc - v) / (k_end - k)
        T = mass * (vn - v) / dt + D + mass * g0 * torch.sin(gamma)
        eta = cf1 * (1.0 + v / cf2)
        fuel = dt * eta * torch.clamp(T, min=0.0)
        xn = x + dt * (v * torch.cos(chi) * torch.cos(gamma) + wx)
        yn = y + dt * (v * torch.sin(chi) * torch.cos(gamma) + wy)
        zn = z + dt * v * torch.sin(gamma)
        chin = chi + dt * chidot
        mn = mass - fuel
        x = torch.where(present, xn, x)
        y = torch.where(present, yn, y)
        z = torch.where(present, zn, z)
        v = torch.where(present, vn, v)
        chi = torch.where(present, chin, chi)
        mass = torch.where(present, mn, mass)
        with torch.no_grad():
            conds = _ro.landing_conditions(scen, x.numpy(), y.numpy(), z.numpy(),
                                           v.numpy(), chi.numpy())
            ok = np.logical_and.reduce([lhs <= rhs for lhs, rhs in conds])
            landed = present & is_arr & torch.as_tensor(ok)
        # time-to-go element at the new state
        vv = torch.clamp(v, min=vmin)
        r = torch.sqrt(x * x + y * y)
        tha = torch.abs(torch.atan2(y, x))
        safe = torch.clamp(torch.sin(tha), min=1e-6)
        ratio = torch.where(tha > 1e-4, tha / safe, 1.0 + tha * tha / 6.0)
        t_arr = torch.clamp(r * ratio / vv / scen["time_norm"], max=1.0)
        t_dep = torch.clamp(torch.clamp(dtma - r, min=0.0) / vv / scen["time_norm"], max=1.0)
        tt = torch.where(is_arr, t_arr, t_dep)
        acc_t = acc_t + torch.where(present & ~landed, tt, torch.zeros_like(tt))
        done = done | landed
    w = scen["cost_w"]
    mix = 1.0 - w[7] - w[8]
    a_fuel = torch.where(is_arr, torch.tensor(w[2], dtype=f64), torch.tensor(w[4], dtype=f64))
    denom = dt * torch.clamp(n_steps, min=1) * tmax * (cf1 * (1.0 + vmax / cf2))
    fuel_term = (m_act - mass) / denom
    ft = mix * a_fuel * fuel_term + w[7] * acc_t / torch.clamp(n_steps, min=1)
    return torch.where(active, ft, torch.zeros_like(ft))


def grad_fuel_time(scen, u_norm, W, states=None, k_active=None, horizon=None):
    """d/du of sum_i c_hat_i^{fuel+time} (mean over the M samples) for every
    particle: returns (value [L, N], gradient [L, N, S, 3])."""
    import torch
    u = torch.tensor(np.asarray(u_norm, dtype=np.float64), requires_grad=True)
    ft = fuel_time_torch(scen, u, W, states, k_active, horizon)
    chat = ft.mean(dim=1)
    chat.sum().backward()
    return chat.detach().numpy(), u.grad.detach().numpy()


# --- the Langevin move in logit coordinates ---------------------------------
# The controls live in the box (0, 1)^D under a uniform prior (Sec.
# "Particles").  The move runs on theta = logit(u), which maps the box onto
# R^D one-to-one, so no proposal can leave the box.  Carried to theta, the
# tempered target exp(-beta sum_i c_hat_i) on the box gains the Jacobian of
# u = logistic(theta), prod_d u_d (1 - u_d); its log-gradient in theta is
#   g u (1 - u) + 1 - 2 u,   g = -beta grad_u sum_i c_hat_i,
# and the proposal is theta' = theta + (eps^2 / 2) (that gradient) + eps xi:
# eps is a standard deviation in logit units.

def logit(u):
    return np.log(u) - np.log1p(-u)


def logistic(t):
    e = np.exp(-np.abs(t))
    return np.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def log_jacobian(u):
    """log prod_d u_d (1 - u_d) per particle: log |du / dtheta|."""
    lj = np.log(u) + np.log1p(-u)
    return np.sum(lj.reshape(lj.shape[0], -1), axis=1)


def mala_drift(u, g, eps):
    """(eps^2 / 2) times the log-gradient in theta of the target carried to
    logit coordinates, at u = logistic(theta), from g (the gradient in u)."""
    return 0.5 * eps * eps * (g * u * (1.0 - u) + 1.0 - 2.0 * u)


def mala_log_q(u_to, u_from, g_from, eps):
    """log q(theta_to | theta_from) up to a constant, per particle: the
    Gaussian N(theta_from + drift(u_from), eps^2 I) of the Langevin proposal
    in logit coordinates."""
    d = logit(u_to) - logit(u_from) - mala_drift(u_from, g_from, eps)
    return -np.sum(d.reshape(d.shape[0], -1) ** 2, axis=1) / (2.0 * eps * eps)
