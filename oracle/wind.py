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


def cholesky_lower(K):
    """Textbook (row by row) Cholesky factorisation K = L L^T, FP64.

    The 1-D squared-exponential Gram matrices are nearly singular, so their
    factors are sensitive to rounding; a fixed, explicit operation order
    keeps this factor reproducible."""
    n = K.shape[0]
    L = np.zeros((n, n))
    for j in range(n):
        s = K[j, j]
        for k in range(j):
            s -= L[j, k] * L[j, k]
        if not s > 0.0:
            raise np.linalg.LinAlgError("matrix not positive definite")
        d = math.sqrt(s)
        L[j, j] = d
        for i in range(j + 1, n):
            t = K[i, j]
            for k in range(j):
                t -= L[i, k] * L[j, k]
            L[i, j] = t / d
    return L


def axis_factor(nodes, ell, nugget):
    """Lower Cholesky factor of the 1-D Gram matrix plus the nugget."""
    K = se_gram(nodes, ell)
    for a in range(len(nodes)):
        K[a, a] += nugget
    return cholesky_lower(K)


def kron_factor(box, grid_n, sigma, ell, nugget):
    """Dense G x G factor L = sigma * Lx (x) Ly (x) Lz.

    Grid point g = (ix * ny + iy) * nz + iz (z fastest), which is the index
    order of the Kronecker product."""
    ax, ay, az = grid_axes(box, grid_n)
    Lx, Ly, Lz = (axis_factor(a, ell, nugget) for a in (ax, ay, az))
    return sigma * np.kron(np.kron(Lx, Ly), Lz)


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
    """The wind fields W_J[m, g, c] of one SMC iteration."""
    if Lfac is None:
        Lfac = kron_factor(scen["box"], scen["grid"], scen["wind_sigma"],
                           scen["wind_ell"], scen["wind_nugget"])
    step = scen["mpc_step"] if mpc_step is None else mpc_step
    G = int(np.prod(scen["grid"]))
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
