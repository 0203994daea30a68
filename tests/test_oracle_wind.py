"""Pins of the oracle's wind model (Sec. "Wind Model")."""
import numpy as np

from oracle import wind

BOX = (60e3, 60e3, 6e3)


def _points(box, grid_n):
    ax, ay, az = wind.grid_axes(box, grid_n)
    X, Y, Z = np.meshgrid(ax, ay, az, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def test_kronecker_factor_reproduces_3d_se_covariance():
    """L L^T equals sigma^2 exp(-|p - q|^2 / 2 ell^2) evaluated directly on
    the 3-D grid points (so the grid index order must match the Kronecker
    order), up to the nugget."""
    grid_n, sigma, ell, d = (6, 5, 3), 5.0, 20e3, 1e-10
    Lf = wind.kron_factor(BOX, grid_n, sigma, ell, d)
    P = _points(BOX, grid_n)
    D2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    R = sigma ** 2 * np.exp(-D2 / (2 * ell ** 2))
    err = np.abs(Lf @ Lf.T - R).max()
    assert err <= 3 * d * sigma ** 2 * 1.01 + 1e-12
    assert np.allclose(Lf, np.tril(Lf))


def test_field_statistics():
    grid_n = (4, 4, 2)
    G = 32
    scen = dict(box=np.array(BOX), grid=np.array(grid_n), wind_sigma=5.0,
                wind_ell=20e3, wind_nugget=1e-10, seed=3, mpc_step=0, M=4000,
                wind_mean=np.array([2.0, -1.0]))
    W = wind.sample_field(scen, J=0)
    assert W.shape == (4000, G, 2)
    assert np.allclose(W[..., 0].mean(0), 2.0, atol=0.3)
    assert np.allclose(W[..., 1].mean(0), -1.0, atol=0.3)
    P = _points(BOX, grid_n)
    C = np.cov(W[..., 0].T)
    D2 = ((P[:, None, :] - P[None, :, :]) ** 2).sum(-1)
    R = 25.0 * np.exp(-D2 / (2 * 20e3 ** 2))
    assert np.abs(C - R).max() < 2.5          # ~4 sigma for 4000 samples
    # the two components are independent
    Cxy = np.mean((W[..., 0] - 2.0) * (W[..., 1] + 1.0), axis=0)
    assert np.abs(Cxy).max() < 1.6


def test_trilinear_exact_on_affine_fields_and_nodes():
    grid_n = (5, 4, 3)
    P = _points(BOX, grid_n)
    a = np.array([1.5, -0.5])
    B = np.array([[1e-4, 2e-4, -3e-3], [-2e-4, 5e-5, 1e-3]])
    W = (a[None, :] + P @ B.T)[None]               # one sample
    rng = np.random.default_rng(0)
    x = rng.uniform(-30e3, 30e3, 1000)
    y = rng.uniform(-30e3, 30e3, 1000)
    z = rng.uniform(0, 6e3, 1000)
    out = wind.trilinear(W, 0, BOX, grid_n, x, y, z)
    exp = a[None, :] + np.stack([x, y, z], 1) @ B.T
    assert np.allclose(out, exp, rtol=0, atol=1e-12)
    # at nodes: node values (including the last node of each axis)
    Wr = rng.normal(size=(1, len(P), 2))
    out = wind.trilinear(Wr, 0, BOX, grid_n, P[:, 0], P[:, 1], P[:, 2])
    assert np.allclose(out, Wr[0], atol=1e-13)
    # clamping outside the grid: equal to the value at the nearest face
    out_far = wind.trilinear(W, 0, BOX, grid_n, np.array([1e6]), np.array([0.0]),
                             np.array([-50.0]))
    out_face = wind.trilinear(W, 0, BOX, grid_n, np.array([30e3]), np.array([0.0]),
                              np.array([0.0]))
    assert np.allclose(out_far, out_face)
