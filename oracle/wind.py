"""Wind disturbance: grid, Gaussian field samples, trilinear interpolation.

Test infrastructure (CPU oracle); never part of the product path.

Paper, Sec. "Wind Model": the wind error is a zero-mean Gaussian random field
on an Nx x Ny x Nz grid; the two horizontal components are independent and
share one covariance matrix R-hat over the grid points; samples are drawn as
(Cholesky factor of R-hat) x (standard normal vector); the wind at an aircraft
is the trilinear interpolation of the grid values; a nominal (forecast) wind is
added to the stochastic part.

Readings used here (listed with the others in the design notes):
  * covariance: squared-exponential per axis with one length scale ell,
    R = sigma^2 Kx (x) Ky (x) Kz (Kronecker product), in place of the paper's
    exponential kernel with a time term;
  * factor: L = sigma Lx (x) Ly (x) Lz with L_a = chol(K_a + delta I),
    delta = 1e-10, so that L L^T = sigma^2 (Kx+dI)(x)(Ky+dI)(x)(Kz+dI);
  * one static field per wind sample, drawn afresh every SMC iteration (the
    paper samples new disturbances on every pass of the inner loop);
  * outside the grid, coordinates are clamped to the grid.

The paper's own model is also here (wind_model 1): the exponential
covariance of the "Wind Model" section, sigma^2 exp(-beta |dxy|) exp(-gamma
|dz|) with the Euclidean horizontal distance, and the linear Gaussian time
recursion W(0) = Qhat v(0), W(k+1) = a W(k) + Q v(k+1) with Qhat Qhat^T =
R-hat, Q Q^T = (1 - a^2) R-hat and a = exp(-dt / G_t): one field per step of
the horizon.  Its readings: sigma(z) is constant; the factor is taken as
sigma L_h (x) L_z, L_h = chol(R_h + delta I) over the nx ny horizontal nodes
and L_z = chol(R_z + delta I) over the nz levels (the covariance is a
Kronecker product of the two, so this is the Cholesky factor of R-hat); the
step-k normals of sample m are those of the static model's sample k M + m.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox


def _nodes(lo, hi, n):
    """n evenly spaced nodes lo + (hi - lo) a / (n - 1)."""
    return np.array([lo + (hi - lo) * a / (n - 1) for a in range(n)])


def grid_axes(box, grid_n):
    """Node coordinates: x, y in [-W/2, W/2], z in [0, Z_top], evenly spaced."""
    wx, wy, zt = (float(b) for b in box)
    nx, ny, nz = (int(n) for n in grid_n)
    return (_nodes(-0.5 * wx, 0.5 * wx, nx), _nodes(-0.5 * wy, 0.5 * wy, ny),
            _nodes(0.0, zt, nz))


def se_gram(nodes, ell):
    """K[a, b] = exp(-(p_a - p_b)^2 / (2 ell^2))."""
    n = len(nodes)
    K = np.empty((n, n))
    for a in range(n):
        for b in range(n):
            d = nodes[a] - nodes[b]
            K[a, b] = math.exp(-d * d / (2.0 * ell * ell))
    return K


def axis_factor(nodes, ell, nugget):
    """Lower Cholesky factor of the 1-D Gram matrix plus the nugget."""
    K = se_gram(nodes, ell)
    for a in range(len(nodes)):
        K[a, a] += nugget
    return np.linalg.cholesky(K)


def kron_factor(box, grid_n, sigma, ell, nugget):
    """Dense G x G factor L = sigma * Lx (x) Ly (x) Lz.

    Grid point g = (ix * ny + iy) * nz + iz (z fastest), which is the index
    order of the Kronecker product."""
    ax, ay, az = grid_axes(box, grid_n)
    Lx, Ly, Lz = (axis_factor(a, ell, nugget) for a in (ax, ay, az))
    return sigma * np.kron(np.kron(Lx, Ly), Lz)


def exp_gram_h(ax, ay, beta):
    """R_h[p, q] = exp(-beta |(x_p - x_q, y_p - y_q)|) over the horizontal
    nodes p = ix * ny + iy (Euclidean distance, eq. cov)."""
    pts = [(x, y) for x in ax for y in ay]
    n = len(pts)
    K = np.empty((n, n))
    for p in range(n):
        for q in range(n):
            dx, dy = pts[p][0] - pts[q][0], pts[p][1] - pts[q][1]
            K[p, q] = math.exp(-beta * math.sqrt(dx * dx + dy * dy))
    return K


def exp_gram_z(az, gamma):
    """R_z[a, b] = exp(-gamma |z_a - z_b|) over the levels (eq. cov)."""
    n = len(az)
    K = np.empty((n, n))
    for a in range(n):
        for b in range(n):
            K[a, b] = math.exp(-gamma * abs(az[a] - az[b]))
    return K


def exp_factor(box, grid_n, sigma, beta, gamma, nugget):
    """Dense G x G factor Qhat = sigma L_h (x) L_z of the exponential
    covariance (grid point g = (ix * ny + iy) * nz + iz, as kron_factor)."""
    ax, ay, az = grid_axes(box, grid_n)
    Kh = exp_gram_h(ax, ay, beta) + nugget * np.eye(len(ax) * len(ay))
    Kz = exp_gram_z(az, gamma) + nugget * np.eye(len(az))
    return sigma * np.kron(np.linalg.cholesky(Kh), np.linalg.cholesky(Kz))


def ar1_coefficient(dt, tcorr):
    """a = exp(-dt / G_t) of the time recursion."""
    return math.exp(-dt / tcorr)


def ar1_fields(Qhat, V, a, wind_mean):
    """The paper's linear Gaussian model over H steps.

    V[k] (H, G, M, 2): the standard normals of step k.  W(0) = Qhat v(0),
    W(k+1) = a W(k) + Q v(k+1), Q = sqrt(1 - a^2) Qhat; the nominal wind is
    added to every step's field.  Returns W[k, m, g, c] (H, M, G, 2)."""
    H, G, M, _ = V.shape
    Q = math.sqrt(1.0 - a * a) * Qhat
    out = np.empty((H, M, G, 2))
    Wk = None
    for k in range(H):
        vk = V[k].reshape(G, M * 2)
        Wk = Qhat @ vk if k == 0 else a * Wk + Q @ vk
        out[k] = Wk.reshape(G, M, 2).transpose(1, 0, 2)
    out += np.asarray(wind_mean, dtype=np.float64)[None, None, None, :]
    return out


def ar1_normals(seed, mpc_step, J, G, M, H, scenario=0):
    """V[k, g, m, c]: the normals of step k, sample m are those the static
    model draws for sample k M + m."""
    Z = wind_normals(seed, mpc_step, J, G, H * M, scenario)
    return Z.reshape(G, H, M, 2).transpose(1, 0, 2, 3).copy()


def factor(scen):
    """The dense factor of the scenario's wind model."""
    if int(scen.get("wind_model", 0)) == 1:
        return exp_factor(scen["box"], scen["grid"], scen["wind_sigma"],
                          scen["wind_beta"], scen["wind_gamma"], scen["wind_nugget"])
    return kron_factor(scen["box"], scen["grid"], scen["wind_sigma"],
                       scen["wind_ell"], scen["wind_nugget"])


def wind_normals(seed, mpc_step, J, G, M, scenario=0):
    """Standard normals Z[g, m, c] for grid point g, sample m, component c.

    One Philox counter per (m, g), element index e = m * G + g; the
    Box-Muller pair gives c = 0 (x, east) and c = 1 (y, north)."""
    e = np.arange(M * G, dtype=np.int64)
    z0, z1 = philox.normals_pair(seed, mpc_step, J, philox.WIND, e, scenario)
    Z = np.empty((G, M, 2))
    Z[:, :, 0] = z0.reshape(M, G).T
    Z[:, :, 1] = z1.reshape(M, G).T
    return Z


def wind_field(Lfac, Z, wind_mean):
    """W[m, g, c] = wbar_c + sum_h L[g, h] Z[h, m, c]."""
    G, M, _ = Z.shape
    W = Lfac @ Z.reshape(G, M * 2)
    W = W.reshape(G, M, 2).transpose(1, 0, 2).copy()
    W += np.asarray(wind_mean, dtype=np.float64)[None, None, :]
    return W


def sample_field(scen, J, mpc_step=None, Lfac=None):
    """The wind fields of one SMC iteration: W_J[m, g, c] (static model) or
    W_J[k, m, g, c] for the H steps of the horizon (the paper's model)."""
    if Lfac is None:
        Lfac = factor(scen)
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    G = int(np.prod(scen["grid"]))
    if int(scen.get("wind_model", 0)) == 1:
        V = ar1_normals(scen["seed"], step, J, G, scen["M"], scen["H"],
                        scen.get("scenario_id", 0))
        return ar1_fields(Lfac, V, ar1_coefficient(scen["dt"], scen["wind_tcorr"]),
                          scen["wind_mean"])
    Z = wind_normals(scen["seed"], step, J, G, scen["M"],
                     scen.get("scenario_id", 0))
    return wind_field(Lfac, Z, scen["wind_mean"])


def trilinear(W, m, box, grid_n, x, y, z):
    """Trilinear interpolation of the fields W[m, g, c] at points (x, y, z).

    ``m`` (sample index) broadcasts against x, y, z; returns (..., 2).  Each
    coordinate is clamped to the grid, the cell index to [0, n - 2]."""
    wx, wy, zt = (float(b) for b in box)
    nx, ny, nz = (int(n) for n in grid_n)
    fx = np.clip((x + wx / 2) / (wx / (nx - 1)), 0.0, nx - 1)
    fy = np.clip((y + wy / 2) / (wy / (ny - 1)), 0.0, ny - 1)
    fz = np.clip(z / (zt / (nz - 1)), 0.0, nz - 1)
    ix = np.minimum(np.floor(fx).astype(np.int64), nx - 2)
    iy = np.minimum(np.floor(fy).astype(np.int64), ny - 2)
    iz = np.minimum(np.floor(fz).astype(np.int64), nz - 2)
    tx, ty, tz = fx - ix, fy - iy, fz - iz
    out = np.zeros(np.shape(x) + (2,))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                wgt = ((tx if a else 1 - tx) * (ty if b else 1 - ty)
                       * (tz if c else 1 - tz))
                g = ((ix + a) * ny + (iy + b)) * nz + (iz + c)
                out += wgt[..., None] * W[m, g]
    return out
