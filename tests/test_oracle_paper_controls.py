"""Pins of the oracle's rollout under the paper's own control
parametrisation (Sec. "Trajectory Planning and Disturbance Realisations",
eq. (hor); Sec. "Particles"): per-step thrust T, flight-path angle gamma and
bank phi, with v' = v + dt ((T - D)/m - g sin gamma),
chi' = chi + dt L sin(phi) / (m v), L = m g cos(gamma) / cos(phi).

Every check is a closed form of the point-mass model, not a retyping of the
update: steady level flight with thrust equal to drag, the coordinated-turn
radius v^2 / (g tan phi) (the Euler track is a regular polygon whose
circumradius tends to it), the energy of an unpowered drag-free glide (the
explicit Euler drift of 1/2 v^2 + g z is exactly dt^2 g^2 sin^2(gamma) / 2 per
step), and the load factor 1 / cos(phi) of a level turn multiplying the
induced drag by n^2."""
import math

import numpy as np
import pytest

from oracle import rollout as ro
from tests.oracle_helpers import DEG, mini, zero_field

G0 = 9.80665


def _scen(H=40, dt=5.0, v=200.0, chi=0.3, z=3000.0, cd0=0.025, cd2=0.0, m0=60e3):
    s = mini(N=1, H=H, S=H, dt=dt, states=[[1000.0, -2000.0, z, v, chi, m0]],
             control_model=1)
    s["ctrl_lo"] = np.array([0.0, -6 * DEG, -30 * DEG])
    s["ctrl_hi"] = np.array([1.0, 6 * DEG, 30 * DEG])
    s["aircraft"][:, 1] = cd0
    s["aircraft"][:, 2] = cd2
    return s


def _norm(s, T, gamma, phi):
    """Normalised per-step controls [1, 1, H, 3] for physical (T, gamma, phi)."""
    H = s["H"]
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    phys = np.array([T / s["aircraft"][0, 5], gamma, phi])
    u = (phys - lo) / (hi - lo)
    return np.broadcast_to(u, (1, 1, H, 3)).copy()


def _drag0(s, v, z):
    Sw, cd0 = s["aircraft"][0, 0], s["aircraft"][0, 1]
    return 0.5 * ro.isa_density(np.array(z)) * v * v * Sw * cd0


def test_level_flight_with_thrust_equal_to_drag():
    """C_D2 = 0, gamma = phi = 0, T = D: speed, heading and altitude stay,
    the track is a straight line, and the fuel is eta(v) T per second."""
    s = _scen()
    v, chi, z, H, dt = 200.0, 0.3, 3000.0, 40, 5.0
    D = float(_drag0(s, v, z))
    r = ro.rollout(s, _norm(s, D, 0.0, 0.0), zero_field(s), record=True)
    f = r["final"][0, 0, 0]
    assert f[3] == pytest.approx(v, abs=1e-9)
    assert f[4] == pytest.approx(chi, abs=1e-12) and f[2] == pytest.approx(z, abs=1e-9)
    assert f[0] == pytest.approx(1000.0 + H * dt * v * math.cos(chi), rel=1e-11)
    assert f[1] == pytest.approx(-2000.0 + H * dt * v * math.sin(chi), rel=1e-11)
    cf1, cf2 = s["aircraft"][0, 3], s["aircraft"][0, 4]
    assert 60e3 - f[5] == pytest.approx(H * dt * cf1 * (1 + v / cf2) * D, rel=1e-11)
    assert r["feas"].all()


def test_coordinated_turn_radius():
    """Level turn at bank phi, thrust = drag (C_D2 = 0, so drag does not
    change with bank): the heading turns by dt g tan(phi) / v per step and the
    positions are the vertices of a regular polygon with side dt v, whose
    circumradius (dt v / 2) / sin(dchi / 2) tends to v^2 / (g tan phi)."""
    s = _scen(H=60, dt=2.0)
    v, z, phi, dt = 200.0, 3000.0, 25 * DEG, 2.0
    D = float(_drag0(s, v, z))
    r = ro.rollout(s, _norm(s, D, 0.0, phi), zero_field(s), record=True)
    tr = r["track"][:, 0, 0, 0]
    dchi = dt * G0 * math.tan(phi) / v
    assert np.allclose(np.diff(tr[:, 4]), dchi, rtol=1e-12, atol=0)
    p = tr[:, :2]
    # circumcentre of the first three vertices; every vertex on that circle
    (x1, y1), (x2, y2), (x3, y3) = p[0], p[1], p[2]
    d = 2 * (x1 * (y2 - y3) + x2 * (y3 - y1) + x3 * (y1 - y2))
    cx = ((x1 ** 2 + y1 ** 2) * (y2 - y3) + (x2 ** 2 + y2 ** 2) * (y3 - y1)
          + (x3 ** 2 + y3 ** 2) * (y1 - y2)) / d
    cy = ((x1 ** 2 + y1 ** 2) * (x3 - x2) + (x2 ** 2 + y2 ** 2) * (x1 - x3)
          + (x3 ** 2 + y3 ** 2) * (x2 - x1)) / d
    rad = np.hypot(p[:, 0] - cx, p[:, 1] - cy)
    R_poly = (dt * v / 2) / math.sin(dchi / 2)
    assert np.allclose(rad, R_poly, rtol=1e-9)
    R_turn = v * v / (G0 * math.tan(phi))
    assert abs(R_poly / R_turn - 1) < dchi * dchi / 20      # (x/2)/sin(x/2) - 1 ~ x^2/24


def test_unpowered_glide_energy_drift_is_the_euler_term():
    """No drag, no thrust, constant gamma: the continuous model conserves
    1/2 v^2 + g z; explicit Euler adds exactly dt^2 g^2 sin^2(gamma) / 2 per
    step, and no fuel is burned."""
    s = _scen(H=30, cd0=0.0, cd2=0.0)
    gamma, dt = -4 * DEG, 5.0
    r = ro.rollout(s, _norm(s, 0.0, gamma, 0.0), zero_field(s), record=True)
    tr = r["track"][:, 0, 0, 0]
    e = 0.5 * tr[:, 3] ** 2 + G0 * tr[:, 2]
    drift = 0.5 * dt * dt * G0 * G0 * math.sin(gamma) ** 2
    assert np.allclose(np.diff(e), drift, rtol=1e-7, atol=1e-9)
    assert np.all(tr[:, 5] == 60e3)
    # the descent rate is v sin(gamma) with the speed of the step
    assert np.allclose(np.diff(tr[:, 2]), dt * tr[:-1, 3] * math.sin(gamma), rtol=1e-12)


def test_load_factor_multiplies_induced_drag():
    """With thrust equal to the level drag at phi = 0, a bank phi adds the
    induced drag of load factor n = 1 / cos(phi): the first step's speed
    change is -dt q S C_D2 C_L0^2 (n^2 - 1) / m."""
    s = _scen(H=2, cd2=0.04)
    v, z, m0, dt, phi = 200.0, 3000.0, 60e3, 5.0, 30 * DEG
    Sw, cd0, cd2 = s["aircraft"][0, :3]
    q = 0.5 * float(ro.isa_density(np.array(z))) * v * v
    CL0 = m0 * G0 / (q * Sw)
    D0 = q * Sw * (cd0 + cd2 * CL0 * CL0)
    r = ro.rollout(s, _norm(s, D0, 0.0, phi), zero_field(s), record=True)
    dv = r["track"][1, 0, 0, 0, 3] - v
    n2 = 1.0 / math.cos(phi) ** 2
    assert dv == pytest.approx(-dt * q * Sw * cd2 * CL0 * CL0 * (n2 - 1) / m0, rel=1e-9)


def test_limits_of_the_paper_controls():
    """A bank beyond the aircraft's limit and a thrust of zero while level at
    low speed (the aircraft decelerates below v_min) are unary violations."""
    s = _scen(H=20)
    s["aircraft"][:, 7] = 20 * DEG                      # bank limit below the control's 30
    r = ro.rollout(s, _norm(s, 50e3, 0.0, 25 * DEG), zero_field(s))
    assert not r["feas"].any()
    s = _scen(H=40, v=115.0, cd0=0.05)
    r = ro.rollout(s, _norm(s, 0.0, 0.0, 0.0), zero_field(s))
    assert not r["feas"].any()


def test_departure_altitude_band_uses_the_path_angle_bound():
    """The reachable-altitude band of the departure altitude element grows
    at v_max sin(gamma_bound) under the flight-path-angle control."""
    s = _scen()
    assert ro.climb_rate_bound(s) == pytest.approx(250.0 * math.sin(6 * DEG))
    s["control_model"] = 0
    assert ro.climb_rate_bound(s) == pytest.approx(30 * DEG)
