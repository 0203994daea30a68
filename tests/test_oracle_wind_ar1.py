"""Pins of the oracle's time-correlated wind model (paper, Sec. "Wind Model":
the exponential covariance eq. cov and the linear Gaussian time recursion).

Each check is fixed by the mathematics, not by the oracle's own code: the
closed-form Cholesky factor of the 1-D exponential kernel (an
Ornstein-Uhlenbeck sequence), the covariance written out entry by entry from
eq. cov, the stationarity of the recursion (every step's field has
covariance R-hat, lag j has a^j R-hat), its a = 1 limit, the Philox element
numbering shared with the static model, and where the rollout reads the
step's field."""
import math

import numpy as np
import pytest

import synth
from oracle import rollout, wind


def _ou_factor(n, rho):
    """Closed form: chol of [rho^|i-j|] is L[i,0] = rho^i,
    L[i,j] = rho^(i-j) sqrt(1 - rho^2) for 1 <= j <= i."""
    L = np.zeros((n, n))
    for i in range(n):
        L[i, 0] = rho ** i
        for j in range(1, i + 1):
            L[i, j] = rho ** (i - j) * math.sqrt(1.0 - rho * rho)
    return L


def test_vertical_gram_is_ou():
    nodes = [0.0, 700.0, 1400.0, 2100.0, 2800.0]
    gamma = 1.5e-4
    L = np.linalg.cholesky(wind.exp_gram_z(nodes, gamma))
    assert np.abs(L - _ou_factor(5, math.exp(-gamma * 700.0))).max() < 1e-13


def test_horizontal_gram_on_a_line_is_ou():
    ax = [-3000.0, -1000.0, 1000.0, 3000.0]
    beta = 2e-4
    L = np.linalg.cholesky(wind.exp_gram_h(ax, [0.0], beta))
    assert np.abs(L - _ou_factor(4, math.exp(-beta * 2000.0))).max() < 1e-13


def test_horizontal_distance_is_euclidean():
    """Diagonal neighbours are sqrt(hx^2 + hy^2) apart, not hx + hy."""
    ax, ay = [0.0, 3000.0], [0.0, 4000.0]
    K = wind.exp_gram_h(ax, ay, 1e-4)
    # p = (ix 0, iy 0) -> index 0; q = (ix 1, iy 1) -> index 1 * 2 + 1 = 3
    assert K[0, 3] == pytest.approx(math.exp(-1e-4 * 5000.0), rel=1e-15)
    assert K[0, 1] == pytest.approx(math.exp(-1e-4 * 4000.0), rel=1e-15)
    assert K[0, 2] == pytest.approx(math.exp(-1e-4 * 3000.0), rel=1e-15)


def test_factor_reproduces_eq_cov():
    """Qhat Qhat^T against sigma^2 exp(-beta |dxy|) exp(-gamma |dz|) written
    out over every pair of grid points (g = (ix ny + iy) nz + iz)."""
    box, grid = (40e3, 30e3, 6e3), (4, 3, 3)
    sigma, beta, gamma = 4.0, 3e-5, 2e-4
    Q = wind.exp_factor(box, grid, sigma, beta, gamma, 0.0)
    nx, ny, nz = grid
    xs = [-box[0] / 2 + box[0] * i / (nx - 1) for i in range(nx)]
    ys = [-box[1] / 2 + box[1] * i / (ny - 1) for i in range(ny)]
    zs = [box[2] * i / (nz - 1) for i in range(nz)]
    G = nx * ny * nz
    R = np.empty((G, G))
    for g in range(G):
        ix, iy, iz = g // (ny * nz), (g // nz) % ny, g % nz
        for h in range(G):
            jx, jy, jz = h // (ny * nz), (h // nz) % ny, h % nz
            dh = math.hypot(xs[ix] - xs[jx], ys[iy] - ys[jy])
            R[g, h] = sigma * sigma * math.exp(-beta * dh) * math.exp(-gamma * abs(zs[iz] - zs[jz]))
    assert np.allclose(Q, np.tril(Q), atol=0.0)
    assert np.abs(Q @ Q.T - R).max() < 1e-12 * sigma * sigma


def _linear_map(Qhat, H, a):
    """The matrix of V -> W (one component, one sample): column (k', g') is
    the response to a unit normal at step k', point g'."""
    G = Qhat.shape[0]
    A = np.zeros((H * G, H * G))
    for kp in range(H):
        for gp in range(G):
            V = np.zeros((H, G, 1, 2))
            V[kp, gp, 0, 0] = 1.0
            W = wind.ar1_fields(Qhat, V, a, (0.0, 0.0))      # [H, 1, G, 2]
            assert np.all(W[..., 1] == 0.0)
            A[:, kp * G + gp] = W[:, 0, :, 0].reshape(H * G)
    return A


def test_recursion_is_stationary_with_geometric_lags():
    box, grid = (20e3, 20e3, 4e3), (2, 2, 2)
    Qhat = wind.exp_factor(box, grid, 3.0, 5e-5, 3e-4, 0.0)
    R = Qhat @ Qhat.T
    H, a = 5, wind.ar1_coefficient(5.0, 40.0)
    A = _linear_map(Qhat, H, a)
    C = A @ A.T
    G = Qhat.shape[0]
    for k in range(H):
        for j in range(H - k):
            blk = C[(k + j) * G:(k + j + 1) * G, k * G:(k + 1) * G]
            assert np.abs(blk - a ** j * R).max() < 1e-12 * np.abs(R).max(), (k, j)


def test_recursion_limit_a_one_is_frozen():
    s = synth.shrink(synth.c1(wind_model="ar1"), M=3, H=4, grid=(3, 3, 2))
    s["wind_tcorr"] = math.inf          # a = exp(-dt / inf) = 1, Q = 0
    W = wind.sample_field(s, J=2)
    assert W.shape == (4, 3, 18, 2)
    for k in range(1, 4):
        assert np.array_equal(W[k], W[0])


def test_step_normals_are_static_samples():
    """Step k, sample m draws the static model's sample k M + m; step 0 is
    the static draw through the same factor."""
    G, M, H = 12, 3, 4
    V = wind.ar1_normals(7, 2, 5, G, M, H)
    Z = wind.wind_normals(7, 2, 5, G, H * M)
    for k in range(H):
        for m in range(M):
            assert np.array_equal(V[k, :, m], Z[:, k * M + m])
    s = synth.shrink(synth.c1(wind_model="ar1"), M=M, H=H, grid=(3, 2, 2))
    Q = wind.factor(s)
    W = wind.sample_field(s, J=1)
    W0 = wind.wind_field(Q, wind.wind_normals(s["seed"], s["mpc_step"], 1, G, M), s["wind_mean"])
    assert np.abs(W[0] - W0).max() < 1e-12


def test_rollout_reads_the_field_of_its_step():
    """A uniform east wind c present at step k0 only moves x by dt c from
    step k0 + 1 on (the Euler update adds the wind at the current step)."""
    s = synth.shrink(synth.c1(wind_model="ar1"), M=1, H=12, S=3, grid=(2, 2, 2))
    rng = np.random.default_rng(1)
    u = rng.uniform(0.3, 0.7, (1, s["N"], s["S"], 3))
    G = 8
    W0 = np.zeros((s["H"], 1, G, 2))
    k0, c = 5, 7.0
    W1 = W0.copy()
    W1[k0, :, :, 0] = c
    t0 = rollout.rollout(s, u, W0, record=True)["track"][:, 0, 0]
    t1 = rollout.rollout(s, u, W1, record=True)["track"][:, 0, 0]
    d = t1[:, :, 0] - t0[:, :, 0]                      # [H + 1, N] x shift
    moving = s["k_active"] <= k0
    assert np.all(d[:k0 + 1] == 0.0)
    assert np.allclose(d[k0 + 1:, moving], s["dt"] * c, rtol=0, atol=1e-9)
    # a field constant in time is the static model
    Ws = rng.normal(size=(1, G, 2))
    r3 = rollout.rollout(s, u, Ws)
    r4 = rollout.rollout(s, u, np.broadcast_to(Ws, (s["H"],) + Ws.shape).copy())
    assert np.array_equal(r3["cost"], r4["cost"]) and np.array_equal(r3["feas"], r4["feas"])
