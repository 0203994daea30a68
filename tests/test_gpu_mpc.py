"""GPU parity of the receding-horizon loop (Sec. "Model Predictive Control",
"Rolling Window"): the plant step against the oracle's, and whole loops of
MPC updates against the oracle's loop."""
import math

import numpy as np
import pytest

import synth
from oracle import mpc as ompc
from tests.gpu_helpers import rel_err

pytestmark = pytest.mark.gpu


def _plan(s, rng):
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    u = rng.uniform(0.2, 0.8, (s["N"], s["S"], 3))
    return lo + u * (hi - lo)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("n_steps", [1, 10, 23])
def test_plant_step_matches_oracle(lib, prec, n_steps):
    """Ten aircraft (arrivals, departures joining at steps 0, 12, 24, 36),
    random plans, the plant's own wind sample: states, activation steps and
    events against the oracle."""
    s = synth.shrink(synth.c2(precision=prec), M=4, L=8, K=2, H=60, S=6, grid=(8, 8, 4))
    ctx = lib.smc_mpc_init(s)
    rng = np.random.default_rng(n_steps)
    ctrl = _plan(s, rng)
    got = lib.smc_plant_step(ctx, ctrl, plant_iter=5, n_steps=n_steps, mpc_step=3)
    ref = ompc.plant_step(s, ctrl, s["states"], s["k_active"], n_steps, plant_iter=5, mpc_step=3)
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
    st, rs = got[0], ref[0]
    scale = np.array([1e5, 1e5, 1e4, 250.0, 2 * math.pi, 1e5])
    assert (np.abs(st - rs) / scale).max() < tol, (np.abs(st - rs) / scale).max()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_plant_events_still_air(lib, prec):
    """No wind: an arrival on the final approach lands, a departure leaves
    through its exit radius, a late joiner flies its steps after joining,
    one not yet joined keeps its state, an inactive one stays inactive."""
    s = synth.make_scenario("P", n_arr=1, n_dep=4, box=(100e3, 100e3, 8e3), grid=(6, 6, 3),
                            H=30, dt=5.0, S=3, M=2, L=4, K=2, seed=4, precision=prec)
    s = dict(s)
    s["wind_sigma"] = 0.0
    s["wind_mean"] = np.zeros(2)
    dtma = s["targets"][1, 3]
    g = math.tan(3.0 * math.pi / 180)
    st = np.array([[9000.0, 0.0, 9000.0 * g, 125.0, math.pi, 60e3],
                   [-(dtma - 2000.0), 0.0, 3000.0, 200.0, math.pi, 60e3],
                   [0.0, 20e3, 3000.0, 150.0, 0.0, 60e3],
                   [0.0, -20e3, 3000.0, 150.0, 0.0, 60e3],
                   [10e3, 30e3, 3000.0, 150.0, 0.0, 60e3]])
    kact = np.array([0, 0, 3, 14, -1], np.int32)
    ctrl = np.zeros((5, s["S"], 3))
    ctrl[:, :, 1] = st[:, 3][:, None]
    ctrl[0, :, 2] = -125.0 * g
    ctx = lib.smc_mpc_init(s)
    got = lib.smc_plant_step(ctx, ctrl, plant_iter=9, n_steps=10, mpc_step=0, states=st,
                             k_active=kact, wind_mean=s["wind_mean"])
    ref = ompc.plant_step(s, ctrl, st, kact, 10, plant_iter=9, mpc_step=0)
    assert list(got[2]) == list(ref[2]) == [1, 2, 0, 0, 0]
    assert list(got[1]) == list(ref[1]) == [-1, -1, 0, 4, -1]
    assert np.array_equal(got[0][3:], st[3:])
    tol = 1e-10 if prec == "fp64" else 2e-5
    assert np.all(rel_err(got[0][:3], ref[0][:3], floor=1.0) < tol)


def test_plant_step_rejects_bad_arguments(lib):
    s = synth.shrink(synth.c1(), L=4, K=2)
    ctx = lib.smc_mpc_init(s)
    ctrl = np.zeros((s["N"], s["S"], 3))
    for kw in (dict(n_steps=0), dict(n_steps=s["H"] + 1), dict(plant_iter=-1)):
        args = dict(plant_iter=3, n_steps=5)
        args.update(kw)
        with pytest.raises(lib.SmcError):
            lib.smc_plant_step(ctx, ctrl, **args)


def test_rolling_window_c1_matches_oracle(lib):
    """Three receding-horizon updates of C1 in FP64 (solve, apply the first
    control segment to the plant, move the window): each update returns the
    oracle's particle, and the plant states stay with the oracle's."""
    s = synth.shrink(synth.c1(), L=128, K=8)
    ctx = lib.smc_mpc_init(s)
    got = lib.rolling_window(ctx, 3)
    ref = ompc.rolling_window(s, 3)
    for t, (g, r) in enumerate(zip(got, ref)):
        assert np.abs(g["controls"] - r["controls"]).max() < 1e-6 * 250.0, t
        assert np.array_equal(g["k_active"], r["k_active"]) and np.array_equal(g["event"], r["event"])
        assert np.all(rel_err(g["states"], r["states"], floor=1.0) < 1e-8), t


@pytest.mark.parametrize("move", ["jitter", "rwmh"])
def test_rolling_window_c1_warm_start_matches_oracle(lib, move):
    """With the warm start each update after the first starts from the
    previous update's final population moved one control segment earlier:
    three C1 updates in FP64 against the oracle's loop (same controls, same
    plant states); the second update differs from a cold loop's."""
    s = synth.shrink(synth.c1(move=move), L=128, K=6)
    sw = dict(s, warm_start=1)
    got = lib.rolling_window(lib.smc_mpc_init(sw), 3)
    ref = ompc.rolling_window(sw, 3)
    for t, (g, r) in enumerate(zip(got, ref)):
        assert np.abs(g["controls"] - r["controls"]).max() < 1e-6 * 250.0, t
        assert np.array_equal(g["k_active"], r["k_active"]) and np.array_equal(g["event"], r["event"])
        assert np.all(rel_err(g["states"], r["states"], floor=1.0) < 1e-8), t
    cold = lib.rolling_window(lib.smc_mpc_init(s), 2)
    assert np.array_equal(cold[0]["controls"], got[0]["controls"])
    assert not np.array_equal(cold[1]["controls"], got[1]["controls"])


def test_warm_start_fp32_update(lib):
    """FP32, 10 aircraft: the second update of a warm-started context
    differs from a cold context's second update, and its returned cost is
    what the FP64 oracle gives the returned particle on that update's last
    fields (within the FP32 bound)."""
    from oracle import smc as osmc
    s = synth.shrink(synth.c2(), M=8, L=64, K=3, H=60, S=6, grid=(8, 8, 4))
    warm = lib.smc_mpc_init(dict(s, warm_start=1))
    cold = lib.smc_mpc_init(s)
    for ctx in (warm, cold):
        lib.smc_mpc_step(ctx, mpc_step=0)
    gw = lib.smc_mpc_step(warm, mpc_step=1)
    gc = lib.smc_mpc_step(cold, mpc_step=1)
    assert not np.array_equal(gw[0], gc[0])
    lo, hi = s["ctrl_lo"], s["ctrl_hi"]
    u_got = (gw[0] - lo) / (hi - lo)
    rc, _ = osmc.eval_cost(s, u_got[None], s["K"] - 1, mpc_step=1)
    assert abs(float(rc.sum()) - gw[1][0]) <= 1e-4 * max(abs(float(rc.sum())), 1.0)
