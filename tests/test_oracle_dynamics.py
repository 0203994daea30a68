"""Pins of the oracle's rollout: closed forms, the paper's inverse relations,
the landing rule, cost bounds and the printed bearing example."""
import math

import numpy as np
import pytest

from oracle import rollout as ro
from oracle import wind
from tests.oracle_helpers import DEG, const_controls, isa_table, mini, zero_field


def _level_scen(H=60, dt=5.0, v=200.0, chi=0.3, z=0.0, cd2=0.04, wind_mean=(0, 0)):
    s = mini(N=1, H=H, S=1, dt=dt, wind_mean=wind_mean,
             states=[[1000.0, -2000.0, z, v, chi, 60e3]])
    # symmetric bounds around the held speed: u = 0.5 maps exactly to v
    s["ctrl_lo"] = np.array([-3 * DEG, v - 50.0, -15.0])
    s["ctrl_hi"] = np.array([3 * DEG, v + 50.0, 15.0])
    s["aircraft"][:, 2] = cd2
    return s


def test_isa_density_matches_standard_tables():
    # tables are at geometric altitude, the model treats z as geopotential
    # altitude: the two differ by z^2 / R_earth (<= 19 m at 11 km); the
    # tables carry 4-5 significant digits
    for z, rho in isa_table().items():
        dh = z * z / 6.356e6           # geometric minus geopotential [m]
        assert abs(ro.isa_density(np.array(z)) - rho) / rho < 1.3e-4 * dh + 1e-4


def test_straight_level_closed_form():
    s = _level_scen()
    r = ro.rollout(s, const_controls(1, 1, 1), zero_field(s), record=True)
    fx = r["final"][0, 0, 0]
    H, dt, v, chi = 60, 5.0, 200.0, 0.3
    assert fx[0] == pytest.approx(1000.0 + H * dt * v * math.cos(chi), rel=1e-12)
    assert fx[1] == pytest.approx(-2000.0 + H * dt * v * math.sin(chi), rel=1e-12)
    assert fx[2] == 0.0 and fx[3] == v and fx[4] == chi


def test_fuel_equals_flow_times_time_without_induced_drag():
    """C_D2 = 0, level, constant speed: thrust = drag = q S C_D0 for every
    step, so fuel = H dt eta(v) q S C_D0 (fuel-flow x time)."""
    s = _level_scen(cd2=0.0)
    r = ro.rollout(s, const_controls(1, 1, 1), zero_field(s))
    S_w, cd0, _, cf1, cf2 = s["aircraft"][0, :5]
    q = 0.5 * 1.225 * 200.0 ** 2                  # sea-level density
    expected = 60 * 5.0 * cf1 * (1 + 200.0 / cf2) * q * S_w * cd0
    burned = 60e3 - r["final"][0, 0, 0, 5]
    assert burned == pytest.approx(expected, rel=1e-12)


def _riccati_mass(m0, a, b, eta, t):
    """Solution of dm/dt = -eta (a + b m^2)."""
    k = math.sqrt(a / b)
    return k * math.tan(math.atan(m0 / k) - eta * math.sqrt(a * b) * t)


def test_mass_ode_with_induced_drag_converges_first_order():
    errs = []
    for H, dt in ((60, 5.0), (120, 2.5), (240, 1.25)):
        s = _level_scen(H=H, dt=dt)
        r = ro.rollout(s, const_controls(1, 1, 1), zero_field(s))
        S_w, cd0, cd2, cf1, cf2 = s["aircraft"][0, :5]
        q = 0.5 * 1.225 * 200.0 ** 2
        a = q * S_w * cd0
        b = cd2 * 9.80665 ** 2 / (q * S_w)
        eta = cf1 * (1 + 200.0 / cf2)
        exact = _riccati_mass(60e3, a, b, eta, 300.0)
        errs.append(abs(r["final"][0, 0, 0, 5] - exact))
    assert errs[0] < 0.05                          # kg, after ~300 kg burned
    assert 1.8 < errs[0] / errs[1] < 2.2 and 1.8 < errs[1] / errs[2] < 2.2


def test_uniform_wind_adds_exact_displacement():
    s0 = _level_scen()
    s1 = _level_scen(wind_mean=(3.0, -2.0))
    r0 = ro.rollout(s0, const_controls(1, 1, 1), zero_field(s0))
    r1 = ro.rollout(s1, const_controls(1, 1, 1), zero_field(s1))
    d = r1["final"][0, 0, 0, :2] - r0["final"][0, 0, 0, :2]
    assert d == pytest.approx([60 * 5.0 * 3.0, -60 * 5.0 * 2.0], rel=1e-9)
    assert r1["final"][0, 0, 0, 5] == r0["final"][0, 0, 0, 5]


def test_fuel_independent_of_wind_for_departures():
    s = mini(N=2, H=30, S=3, M=5, sigma=5.0,
             states=[[0, 0, 400, 110, math.pi, 65e3], [5e3, 5e3, 1000, 150, 0.0, 60e3]])
    rng = np.random.default_rng(0)
    u = rng.uniform(0.3, 0.7, size=(4, 2, 3, 3))
    W = wind.sample_field(s, 0)
    r = ro.rollout(s, u, W)
    m = r["final"][..., 5]
    assert np.all(m == m[:, :1, :])
    assert not np.all(r["final"][..., 0] == r["final"][:, :1, :, 0])


def test_fuel_estimate_1_round_trip():
    """The paper's Fuel Estimate 1 (inverse dynamics from a track) applied to
    a simulated track recovers the wind at the aircraft and the mass."""
    s = mini(N=2, H=24, S=4, M=2, sigma=5.0, wind_mean=(1.0, -2.0),
             states=[[-20e3, 10e3, 3500, 200, -0.4, 62e3], [0, 0, 400, 110, math.pi, 65e3]])
    rng = np.random.default_rng(2)
    u = rng.uniform(0.2, 0.8, size=(3, 2, 4, 3))
    W = wind.sample_field(s, 0)
    r = ro.rollout(s, u, W, record=True)
    tr, pres = r["track"], r["present"]
    g = 9.80665
    checked = 0
    for k in range(s["H"]):
        for l in range(3):
            for m in range(2):
                for i in range(2):
                    if not pres[k, l, m, i]:
                        continue
                    x, y, z, v, chi, mass = tr[k, l, m, i]
                    x1, y1, z1, v1, chi1, m1 = tr[k + 1, l, m, i]
                    dt = s["dt"]
                    S_w, cd0, cd2, cf1, cf2 = s["aircraft"][i, :5]
                    eta = cf1 * (1 + v / cf2)
                    gam = math.asin((z1 - z) / (dt * v))
                    wx = (x1 - x) / dt - v * math.cos(chi) * math.cos(gam)
                    wy = (y1 - y) / dt - v * math.sin(chi) * math.cos(gam)
                    w_true = wind.trilinear(W, m, s["box"], s["grid"], np.array(x),
                                            np.array(y), np.array(z))
                    assert wx == pytest.approx(w_true[0], abs=1e-7)
                    assert wy == pytest.approx(w_true[1], abs=1e-7)
                    # bank from the heading change (Fuel Estimate 2)
                    phi = math.atan((chi1 - chi) * v / (g * dt))
                    rho = isa_table()[0.0] * (1 - 0.0065 * z / 288.15) ** (g / (287.05287 * 0.0065) - 1)
                    q = 0.5 * rho * v * v
                    CL = mass * g / (q * S_w * math.cos(phi))
                    D = q * S_w * (cd0 + cd2 * CL * CL)
                    T = mass * (v1 - v) / dt + D + mass * g * math.sin(gam)
                    assert m1 == pytest.approx(mass - dt * eta * max(T, 0.0), rel=1e-13)
                    checked += 1
    assert checked > 100


def test_landed_arrival_scores_best_cost_afterwards():
    s = mini(N=1, kinds=[0], H=10, S=1,
             states=[[6000.0, 100.0, 300.0, 120.0, math.pi, 60e3]])
    s["ctrl_lo"] = np.array([-3 * DEG, 70.0, -15.0])
    s["ctrl_hi"] = np.array([3 * DEG, 170.0, 15.0])
    r = ro.rollout(s, const_controls(1, 1, 1), zero_field(s), record=True)
    pres = r["present"][:, 0, 0, 0]
    assert pres[0] and not pres[1:].any()        # lands on the first new state
    w = s["cost_w"]
    S_w, cd0, cd2, cf1, cf2, tmax = s["aircraft"][0, :6]
    burned = 60e3 - r["final"][0, 0, 0, 5]
    fuel_term = burned / (5.0 * 10 * tmax * cf1 * (1 + 250.0 / cf2))
    assert r["cost"][0, 0, 0] == pytest.approx((1 - w[7] - w[8]) * w[2] * fuel_term,
                                               rel=1e-12)


def test_flow_field_reaches_runway_heading_after_arc_length():
    """Following chi_hat = pi + 2 atan2(y, x) from a point arrives at the
    origin heading west after flying s_arc = r |theta| / sin|theta|."""
    for x0, y0 in ((20e3, 5e3), (3e3, 25e3), (-10e3, 12e3), (15e3, -18e3)):
        p = np.array([x0, y0])
        th = abs(math.atan2(y0, x0))
        s_pred = math.hypot(x0, y0) * th / math.sin(th)
        flown, ds = 0.0, 2.0
        while math.hypot(*p) > 20.0:
            def f(q):
                c = math.pi + 2 * math.atan2(q[1], q[0])
                return np.array([math.cos(c), math.sin(c)])
            k1 = f(p); k2 = f(p + ds / 2 * k1); k3 = f(p + ds / 2 * k2); k4 = f(p + ds * k3)
            p = p + ds / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
            flown += ds
            assert flown < 3 * s_pred
        assert flown == pytest.approx(s_pred, abs=25.0)
        head = math.pi + 2 * math.atan2(p[1], p[0])
        assert abs(ro.wrap(head - math.pi)) < 0.02


def test_cost_elements_bounded_and_bearing_example():
    s = mini(N=2, kinds=[0, 1])
    rng = np.random.default_rng(5)
    n = 20000
    x = rng.uniform(-40e3, 40e3, (n, 1)); y = rng.uniform(-40e3, 40e3, (n, 1))
    z = rng.uniform(0, 6e3, (n, 1)); v = rng.uniform(110, 250, (n, 1))
    chi = rng.uniform(-20, 20, (n, 1)); j = rng.integers(1, 60, (n, 1))
    # altitude reachable from the activation altitude within j steps
    z_act = np.clip(z + rng.uniform(-1, 1, (n, 1)) * 15.0 * j * s["dt"], 0, 6e3)
    c = ro.step_cost(s, j, x, y, z, v, chi, z_act)
    assert np.all(c >= 0) and np.all(c <= 1)
    # the printed example: on the desired bearing every step -> best
    # bearing element; 90 degrees off -> half of it
    s2 = mini(N=1, kinds=[1])
    s2["cost_w"] = np.array([0, 0, 0, 1.0, 0, 0, 0, 0, 0])
    thF = s2["targets"][0, 0]
    on = ro.step_cost(s2, 5, 10e3 * math.cos(thF), 10e3 * math.sin(thF), 3000.0,
                      200.0, 0.0, 400.0)
    off = ro.step_cost(s2, 5, 10e3 * math.cos(thF + math.pi / 2),
                       10e3 * math.sin(thF + math.pi / 2), 3000.0, 200.0, 0.0, 400.0)
    assert float(np.ravel(on)[0]) == pytest.approx(0.0, abs=1e-15)
    assert float(np.ravel(off)[0]) == pytest.approx(0.5, abs=1e-15)


def test_noise_term_limits():
    s = mini(N=1, kinds=[1])
    s["cost_w"] = np.array([0, 0, 0, 0, 0, 0, 0, 0, 1.0])
    pd = np.random.default_rng(0).uniform(0, 1, (5, 7)).astype(np.float32)
    s["popdense"] = pd
    s["noise_alt"] = 2000.0
    xs = np.linspace(-30e3, 30e3, 7)
    ys = np.linspace(-30e3, 30e3, 5)
    for iy in range(5):
        for ix in range(7):
            c0 = ro.step_cost(s, 1, xs[ix], ys[iy], 0.0, 200.0, 0.0, 0.0)
            assert float(np.ravel(c0)[0]) == pytest.approx(float(pd[iy, ix]), abs=1e-7)
            c1 = ro.step_cost(s, 1, xs[ix], ys[iy], 2500.0, 200.0, 0.0, 0.0)
            assert float(np.ravel(c1)[0]) == 0.0
