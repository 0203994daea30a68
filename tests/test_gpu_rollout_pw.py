"""GPU parity of the rollouts whose lanes are wind samples of particles
(FP32): particle-per-wave (layout 3, 64 samples of one particle per wave)
and the particle tile (layout 4, 4 particles x 16 samples per wave).  The
wind-independent part of every aircraft's step is computed once per
particle, and only pairs inside the vertical separation get the horizontal
test.  Element-wise against the
FP64 oracle (2e-5 relative per world, feasibility exact away from
thresholds), with the simulated aircraft-steps and pair-test counts exact."""
import numpy as np
import pytest

import synth
from tests.test_gpu_kernels import _compare_rollout, _rollout_case

pytestmark = pytest.mark.gpu

LAYOUTS = [3, 4]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("N,M", [(1, 3), (2, 70), (7, 3), (16, 64), (21, 3), (24, 70), (32, 3),
                                 (33, 5), (40, 70), (41, 3), (48, 128), (49, 3), (63, 5), (64, 66)])
def test_rollout_pw_aircraft_counts(lib, N, M, layout):
    """One to 64 aircraft (both vector halves, every register bucket), one or
    two blocks of 64 samples with a ragged tail, mixed kinds and activation
    steps, inactive aircraft."""
    rng = np.random.default_rng(N)
    n_arr = min(max(1, N // 2), 24)
    s = synth.make_scenario("T", n_arr=n_arr, n_dep=N - n_arr,
                            box=(100e3, 100e3, 8e3), grid=(6, 5, 4), H=30, dt=5.0, S=3,
                            M=M, L=8, K=2, precision="fp32", seed=N)
    k_act = s["k_active"].copy()
    k_act[rng.uniform(size=N) < 0.2] = -1
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=11, seed=N, horizon=27, k_active=k_act,
                                            layout=layout)
    n_near = _compare_rollout(gc, gf, ref, 1)
    assert steps == ref["steps"]
    # a wind-independent margin (thrust, bank, climb, speed, altitude, mass)
    # is the same in all M samples of a particle: one near-threshold particle
    # takes its M worlds out of the strict comparison
    assert n_near <= 0.02 * 11 * M + 2 * M


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("N", [12, 33, 40, 41, 64])
def test_rollout_pw_close_traffic_separation(lib, N, layout):
    """Aircraft packed inside one separation cell at altitudes within a few
    hundred metres: many pairs pass the vertical test and many horizontal
    tests fire, in both vector halves."""
    rng = np.random.default_rng(5)
    s = synth.make_scenario("T", n_arr=0, n_dep=N, box=(60e3, 60e3, 6e3), grid=(4, 4, 3),
                            H=8, dt=5.0, S=2, M=66, L=4, K=2, precision="fp32", seed=1)
    st = np.zeros((N, 6))
    st[:, 0] = rng.uniform(-8e3, 8e3, N)
    st[:, 1] = rng.uniform(-8e3, 8e3, N)
    st[:, 2] = rng.uniform(2000, 2800, N)
    st[:, 3] = 150.0
    st[:, 4] = rng.uniform(-3, 3, N)
    st[:, 5] = 60e3
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=9, states=st, k_active=np.zeros(N, np.int32),
                                            layout=layout)
    n_near = _compare_rollout(gc, gf, ref, 1)
    assert steps == ref["steps"]
    assert n_near <= 0.02 * 9 * 66 + 2 * 66
    assert (~ref["feas"]).mean() > 0.2


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rollout_pw_landed_aircraft_leave_the_airspace(lib, layout):
    """Arrivals queued on the final approach land one after the other at one
    altitude: a landed aircraft is parked and never conflicts again."""
    n, H = 4, 40
    s = synth.make_scenario("Q", n_arr=n, n_dep=0, box=(80e3, 80e3, 6e3), grid=(4, 4, 3),
                            H=H, dt=5.0, S=4, M=2, L=4, K=2, precision="fp32", seed=3)
    s = dict(s)
    s["ctrl_lo"] = np.array([-0.1 * np.pi / 180, 110.0, -0.5])
    s["ctrl_hi"] = np.array([0.1 * np.pi / 180, 128.0, 0.5])
    st = np.zeros((n, 6))
    st[:, 0] = 8.3e3 + 6.5e3 * np.arange(n)
    st[:, 2] = 500.0
    st[:, 3] = 120.0
    st[:, 4] = np.pi
    st[:, 5] = 60e3
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=64, states=st,
                                            k_active=np.zeros(n, np.int32), layout=layout)
    _compare_rollout(gc, gf, ref, 1)
    assert steps == ref["steps"] < 64 * 2 * n * H
    assert ref["feas"].all() and gf.all()


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rollout_pw_noise_term(lib, layout):
    s = synth.shrink(synth.c5(), M=3, H=30, S=3, grid=(8, 8, 4))
    ctx, gc, gf, steps, ref = _rollout_case(lib, s, P=6, layout=layout)
    n_near = _compare_rollout(gc, gf, ref, 1)
    assert steps == ref["steps"]
    assert n_near <= 0.02 * 6 * 3 * 40 + 2 * 3


@pytest.mark.parametrize("layout", LAYOUTS)
def test_rollout_pw_refused_in_fp64(lib, layout):
    s = synth.shrink(synth.c5(precision="fp64"), M=2, H=20, S=2, grid=(4, 4, 3), L=4)
    ctx = lib.smc_mpc_init(s)
    with pytest.raises(lib.SmcError):
        lib.smc_set_rollout_layout(ctx, layout)
