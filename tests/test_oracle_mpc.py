"""Pins of the receding-horizon loop's plant step (Sec. "Model Predictive
Control", "Rolling Window"): closed forms of straight and level flight in
still air, activation and retirement bookkeeping, landing and exit events."""
import math

import numpy as np

import synth
from oracle import mpc


def _still_air(n_arr, n_dep, H=30, S=3, **kw):
    s = synth.make_scenario("P", n_arr=n_arr, n_dep=n_dep, box=(100e3, 100e3, 8e3),
                            grid=(6, 6, 3), H=H, dt=5.0, S=S, M=2, L=4, K=2, seed=4, **kw)
    s = dict(s)
    s["wind_sigma"] = 0.0
    s["wind_mean"] = np.zeros(2)
    return s


def _level(s, v):
    """Plan holding heading, airspeed v and altitude on every segment."""
    c = np.zeros((s["N"], s["S"], 3))
    c[:, :, 1] = v
    return c


def test_applied_steps_is_the_first_segment():
    s = _still_air(1, 1, H=30, S=3)
    assert mpc.applied_steps(s) == 10
    assert mpc.applied_steps(s, horizon=31) == 11


def test_straight_level_flight_closed_form():
    """No wind, zero heading rate and climb, airspeed held: the position
    advances by n dt v (cos chi, sin chi); altitude, speed and heading stay;
    the mass falls by the fuel burnt (positive)."""
    s = _still_air(0, 2)
    st = np.array([[20e3, -5e3, 3000.0, 180.0, 0.3, 70e3],
                   [-10e3, 8e3, 2500.0, 200.0, -2.0, 65e3]])
    kact = np.zeros(2, np.int32)
    n = 10
    ctrl = _level(s, st[:, 3][:, None])
    new, k_new, ev = mpc.plant_step(s, ctrl, st, kact, n, plant_iter=9, mpc_step=0)
    for i in range(2):
        v, chi = st[i, 3], st[i, 4]
        assert math.isclose(new[i, 0], st[i, 0] + n * 5.0 * v * math.cos(chi), rel_tol=1e-12)
        assert math.isclose(new[i, 1], st[i, 1] + n * 5.0 * v * math.sin(chi), rel_tol=1e-12,
                            abs_tol=1e-9)
        assert new[i, 2] == st[i, 2] and new[i, 3] == st[i, 3] and new[i, 4] == st[i, 4]
        assert 0 < st[i, 5] - new[i, 5] < 0.01 * st[i, 5]
    assert list(k_new) == [0, 0] and list(ev) == [0, 0]


def test_activation_and_inactive_aircraft():
    """An aircraft joining at step 3 of a 10-step application flies 7 steps;
    one joining at step 14 keeps its state and joins 10 steps earlier next
    time; an inactive one stays inactive and unchanged."""
    s = _still_air(0, 3)
    st = np.array([[0.0, 0.0, 3000.0, 150.0, 0.0, 60e3]] * 3)
    st[1, 1] = 20e3
    st[2, 1] = -20e3
    kact = np.array([3, 14, -1], np.int32)
    new, k_new, ev = mpc.plant_step(s, _level(s, 150.0), st, kact, 10, plant_iter=9,
                                    mpc_step=0)
    assert math.isclose(new[0, 0], 7 * 5.0 * 150.0, rel_tol=1e-12)
    assert np.array_equal(new[1], st[1]) and np.array_equal(new[2], st[2])
    assert list(k_new) == [0, 4, -1] and list(ev) == [0, 0, 0]


def test_arrival_lands_and_leaves_the_problem():
    """An arrival on the final approach (east of the runway, heading west,
    on the glide slope, slow) meets the landing sector within the applied
    steps: event 1, no longer active."""
    s = _still_air(1, 0)
    z0 = 9000.0 * math.tan(3.0 * math.pi / 180)
    st = np.array([[9000.0, 0.0, z0, 125.0, math.pi, 60e3]])
    ctrl = np.zeros((1, s["S"], 3))
    ctrl[:, :, 1] = 125.0
    ctrl[:, :, 2] = -125.0 * math.tan(3.0 * math.pi / 180)
    new, k_new, ev = mpc.plant_step(s, ctrl, st, np.zeros(1, np.int32), 10, plant_iter=9,
                                    mpc_step=0)
    assert list(ev) == [1] and list(k_new) == [-1]
    assert math.hypot(new[0, 0], new[0, 1]) < 8000.0


def test_departure_leaves_through_the_exit_radius():
    s = _still_air(0, 1)
    dtma = s["targets"][0, 3]
    st = np.array([[-(dtma - 2000.0), 0.0, 3000.0, 200.0, math.pi, 60e3]])
    new, k_new, ev = mpc.plant_step(s, _level(s, 200.0), st, np.zeros(1, np.int32), 10,
                                    plant_iter=9, mpc_step=0)
    assert list(ev) == [2] and list(k_new) == [-1]
    assert math.hypot(new[0, 0], new[0, 1]) >= dtma


def test_straight_level_flight_closed_form_time_correlated_wind():
    """The same closed form holds under the paper's time-correlated wind
    model (Sec. "Wind Model") when the air is still (sigma 0, no mean)."""
    s = _still_air(0, 2, wind_model="ar1")
    st = np.array([[20e3, -5e3, 3000.0, 180.0, 0.3, 70e3],
                   [-10e3, 8e3, 2500.0, 200.0, -2.0, 65e3]])
    n = 10
    new, k_new, ev = mpc.plant_step(s, _level(s, st[:, 3][:, None]), st, np.zeros(2, np.int32),
                                    n, plant_iter=9, mpc_step=0)
    for i in range(2):
        v, chi = st[i, 3], st[i, 4]
        assert math.isclose(new[i, 0], st[i, 0] + n * 5.0 * v * math.cos(chi), rel_tol=1e-12)
        assert math.isclose(new[i, 1], st[i, 1] + n * 5.0 * v * math.sin(chi), rel_tol=1e-12,
                            abs_tol=1e-9)
    assert list(ev) == [0, 0]


def test_plant_flies_each_steps_field_of_sample_zero():
    """Under the time-correlated model with zero decay rates in space
    (beta = gamma = 0: every field is one vector over the whole grid, up to
    the nugget) the plant's displacement over n steps of straight and level
    flight is n dt v (cos chi, sin chi) plus dt times the sum of sample 0's
    wind vectors of steps 0 .. n-1 (Euler: the wind at the start of each
    step).  Using one field for all steps, or another sample, fails."""
    from oracle import wind as owind
    s = dict(_still_air(0, 1, wind_model="ar1"))
    s["wind_sigma"] = 5.0
    s["wind_beta"] = 0.0
    s["wind_gamma"] = 0.0
    s["wind_tcorr"] = 60.0            # a = exp(-dt / G_t): fields change from step to step
    st = np.array([[5e3, 2e3, 3000.0, 190.0, 0.7, 68e3]])
    n = 8
    new, _, _ = mpc.plant_step(s, _level(s, 190.0), st, np.zeros(1, np.int32), n,
                               plant_iter=9, mpc_step=0)
    W = owind.sample_field(s, 9, 0)                       # [H, M, G, 2]
    assert W.ndim == 4
    w = W[:n, 0, 0, :]                                    # sample 0, grid point 0
    assert np.ptp(W[:n, 0], axis=1).max() < 1e-3          # uniform over the grid
    assert np.ptp(w[:, 0]) > 0.1                          # and changing in time
    dx = n * 5.0 * 190.0 * math.cos(0.7) + 5.0 * w[:, 0].sum()
    dy = n * 5.0 * 190.0 * math.sin(0.7) + 5.0 * w[:, 1].sum()
    assert abs(new[0, 0] - (st[0, 0] + dx)) < 0.05
    assert abs(new[0, 1] - (st[0, 1] + dy)) < 0.05
    # a plant that used step 0's field throughout would be off by this much
    assert abs(5.0 * (w[:, 0].sum() - n * w[0, 0])) > 1.0
